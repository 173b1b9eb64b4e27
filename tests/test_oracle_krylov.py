"""Pins of the oracle's RAS preconditioner (eq. (4)) and Krylov solvers."""
import numpy as np
import pytest

import oracle
import synth
from synth import CSR


def _dense_csr(d):
    import scipy.sparse as sp
    m = sp.csr_matrix(d)
    m.sort_indices()
    return CSR(d.shape[0], m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())


def test_ras_single_subdomain_is_global_ilu0():
    A = synth.diffusion3d(6, 5, 4, 1.0, seed=1)
    r = synth.rhs(A.n, 2, 2)
    doms = oracle.ras_setup(A, np.zeros(A.n, dtype=np.int32), 1, overlap=1)
    L, U = oracle.ilu0(A)
    assert np.array_equal(oracle.ras_apply(doms, r), oracle.ilu_apply(L, U, r))


def test_ras_no_overlap_is_block_ilu0():
    A = synth.poisson2d(12, 10)
    owner, _ = synth.subdomain_cuts(A.n, 4, 20, 40, seed=3)
    doms = oracle.ras_setup(A, owner, 4, overlap=0)
    # block ILU(0): ILU(0) of A with the couplings between blocks removed
    Ad = A.to_dense()
    Ab = np.where(owner[:, None] == owner[None, :], Ad, 0.0)
    L, U = oracle.ilu0(_dense_csr(Ab))
    r = synth.rhs(A.n, 1, 4)
    assert np.array_equal(oracle.ras_apply(doms, r), oracle.ilu_apply(L, U, r))


def test_ras_partition_of_unity_and_overlap():
    A = synth.poisson3d(6)
    owner, _ = synth.subdomain_cuts(A.n, 5, 20, 80, seed=5)
    doms = oracle.ras_setup(A, owner, 5, overlap=1)
    owned = np.concatenate([d.owned_global for d in doms])
    assert np.array_equal(np.sort(owned), np.arange(A.n))
    S = A.to_scipy()
    for d in doms:
        nb = np.unique(S[d.owned_global].indices)
        assert np.array_equal(d.ext, np.union1d(d.owned_global, nb))
        assert np.array_equal(d.ext[d.owned_local], d.owned_global)


def test_gmres_exact_preconditioner_one_iteration():
    A = synth.diffusion2d(8, 8, 1.0, seed=6)
    Ad = A.to_dense()
    b = synth.rhs(A.n, 1, 7)[:, 0]
    x, info = oracle.fgmres(A, b, lambda v: np.linalg.solve(Ad, v), m=10, rtol=1e-10)
    assert info.converged and info.iters == 1


def test_gmres_unpreconditioned_finite_termination():
    n = 24
    rng = np.random.default_rng(8)
    Ad = np.eye(n) * 3 + rng.uniform(-1, 1, (n, n)) * 0.5
    A = _dense_csr(Ad)
    b = rng.uniform(-1, 1, n)
    x, info = oracle.fgmres(A, b, lambda v: v, m=n, rtol=1e-12)
    assert info.converged and info.iters <= n
    assert np.allclose(x, np.linalg.solve(Ad, b), rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("solver", ["gmres", "gmres_restarted", "bicgstab"])
def test_ilu0_preconditioned_solves_reach_tolerance(solver):
    A = synth.poisson3d(12)
    L, U = oracle.ilu0(A)
    b = synth.rhs(A.n, 1, 9)[:, 0]

    def M(v):
        return oracle.ilu_apply(L, U, v)

    if solver == "gmres":
        x, info = oracle.fgmres(A, b, M, m=30, rtol=1e-10)
    elif solver == "gmres_restarted":
        x, info = oracle.fgmres(A, b, M, m=4, rtol=1e-10)
    else:
        x, info = oracle.bicgstab(A, b, M, rtol=1e-10)
    assert info.converged
    true = np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)
    assert true <= 1e-10 and abs(true - info.relres) <= 1e-14
    xe = np.linalg.solve(A.to_dense(), b)
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) < 1e-8


def test_mixed_precision_refinement_reaches_fp64_tolerance():
    A = synth.diffusion3d(10, 10, 10, 2.0, seed=3)
    L, U = oracle.ilut(A, 10, 1e-3)
    L32, U32 = oracle.to_f32(L), oracle.to_f32(U)
    b = synth.rhs(A.n, 1, 3)[:, 0]
    x64, i64 = oracle.fgmres(A, b, lambda v: oracle.ilu_apply(L, U, v), m=30, rtol=1e-10)
    x32, i32 = oracle.fgmres(A, b, lambda v: oracle.ilu_apply_f32(L32, U32, v), m=30, rtol=1e-10)
    assert i64.converged and i32.converged
    assert i32.relres <= 1e-10
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) < 1e-7


def test_ras_preconditioned_bicgstab():
    A = synth.poisson3d(10)
    owner, _ = synth.subdomain_cuts(A.n, 4, 150, 400, seed=4)
    doms = oracle.ras_setup(A, owner, 4, overlap=1)
    d32 = oracle.ras_to_f32(doms)
    b = synth.rhs(A.n, 1, 4)[:, 0]
    x, info = oracle.bicgstab(A, b, lambda v: oracle.ras_apply_f32(d32, v), rtol=1e-10)
    assert info.converged and info.relres <= 1e-10


@pytest.mark.parametrize("kind,args", [("iluk", {"k": 1}), ("iluk", {"k": 2}),
                                       ("ilut", {"p": 7, "tau": 0.1}), ("ilut", {"p": 10, "tau": 1e-3})])
def test_block_ilu_is_the_factorization_of_the_decoupled_matrix(kind, args):
    # block ILU(k) / block ILUT (Section 3, overlap 0): the same factorization
    # applied to A with every coupling between blocks removed
    A = synth.diffusion3d(8, 7, 6, 1.0, seed=12)
    owner = synth.grid_bisection(8, 7, 6, 5)
    doms = oracle.ras_setup(A, owner, 5, overlap=0, kind=kind, **args)
    Ad = A.to_dense()
    Ab = _dense_csr(np.where(owner[:, None] == owner[None, :], Ad, 0.0))
    L, U = oracle.iluk(Ab, args["k"]) if kind == "iluk" else oracle.ilut(Ab, args["p"], args["tau"])
    r = synth.rhs(A.n, 2, 13)
    assert np.array_equal(oracle.ras_apply(doms, r), oracle.ilu_apply(L, U, r))


def test_block_ilut_without_dropping_is_the_exact_block_solve():
    # tau = 0 and p >= block size keeps every entry: each block is solved exactly
    A = synth.diffusion2d(9, 8, 1.5, seed=14)
    owner = synth.grid_bisection(9, 8, 1, 4)
    doms = oracle.ras_setup(A, owner, 4, overlap=0, kind="ilut", tau=0.0, p=A.n)
    Ab = np.where(owner[:, None] == owner[None, :], A.to_dense(), 0.0)
    r = synth.rhs(A.n, 1, 15)
    ref = np.linalg.solve(Ab, r)
    assert np.linalg.norm(oracle.ras_apply(doms, r) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_grid_bisection_boxes():
    owner = synth.grid_bisection(10, 9, 7, 12)
    sizes = np.bincount(owner)
    assert len(sizes) == 12 and sizes.sum() == 630
    o = owner.reshape(7, 9, 10)
    for s in range(12):
        z, y, x = np.nonzero(o == s)
        box = (z.max() - z.min() + 1) * (y.max() - y.min() + 1) * (x.max() - x.min() + 1)
        assert box == sizes[s]  # every part is one axis-aligned box
    with pytest.raises(ValueError):
        oracle.ras_setup(synth.poisson2d(4), np.zeros(16, np.int32), 1, kind="ilu2")
