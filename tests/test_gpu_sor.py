"""GPU parity of the SOR / Gauss-Seidel smoother (Section 1's Gauss-Seidel
smoothers, built on the level-scheduled lower and upper solves of
Algorithm 2) against the oracle's elementwise sweeps."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1606_00541_amd as H  # noqa: E402
from parity import relerr  # noqa: E402  (normwise and element-wise)

TOL = 1e-12




@pytest.mark.parametrize("omega", [1.0, 0.8, 1.3])
@pytest.mark.parametrize("symmetric", [False, True])
@pytest.mark.parametrize("nrhs,sweeps", [(1, 1), (3, 4)])
def test_sor_matches_oracle(omega, symmetric, nrhs, sweeps):
    A = synth.diffusion3d(17, 15, 13, 1.5, seed=21)
    s = H.sor_setup(A, omega, tune=H.tune_default(max_nrhs=nrhs))
    b = synth.rhs(A.n, nrhs, 22)
    x0 = synth.rhs(A.n, nrhs, 23)
    xt = torch.from_numpy(x0.copy()).cuda()
    H.sor_apply(s, torch.from_numpy(b).cuda(), xt, sweeps=sweeps, symmetric=symmetric)
    ref = oracle.sor(A, b, x0, omega=omega, sweeps=sweeps, symmetric=symmetric)
    assert relerr(xt.cpu().numpy(), ref) <= TOL


def test_sor_nonsymmetric_pattern_and_zero_sweeps():
    # a random sparse matrix with unsymmetric pattern and long-range couplings
    T = synth.random_lower(900, 0.004, 31)
    M = T.to_scipy() + synth.random_lower(900, 0.004, 32).to_scipy().T
    M = M.tocsr()
    M.sort_indices()
    A = synth.CSR(900, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.copy())
    s = H.sor_setup(A, 1.1)
    b = synth.rhs(900, 2, 33)
    x0 = synth.rhs(900, 2, 34)
    xt = torch.from_numpy(x0.copy()).cuda()
    bt = torch.from_numpy(b).cuda()
    H.sor_apply(s, bt, xt, sweeps=0)
    assert np.array_equal(xt.cpu().numpy(), x0)
    H.sor_apply(s, bt, xt, sweeps=2, symmetric=True)
    assert relerr(xt.cpu().numpy(), oracle.sor(A, b, x0, omega=1.1, sweeps=2, symmetric=True)) <= TOL
    with pytest.raises(H.HecError):
        H.sor_apply(s, xt, xt)


def test_gauss_seidel_converges_on_poisson():
    A = synth.poisson3d(20)
    s = H.sor_setup(A, 1.0)
    b = synth.rhs(A.n, 1, 35)
    xt = torch.zeros(A.n, 1, dtype=torch.float64, device="cuda")
    H.sor_apply(s, torch.from_numpy(b).cuda(), xt, sweeps=400, symmetric=True)
    x = xt.cpu().numpy()[:, 0]
    assert np.linalg.norm(b[:, 0] - oracle.spmv(A, x)) / np.linalg.norm(b[:, 0]) <= 1e-8
