"""Pins of the oracle's SOR / Gauss-Seidel sweeps (the smoothers Section 1
names among the users of triangular solves): the matrix form of a sweep, the
one-sweep exact solve of a triangular system, and the energy-norm decrease
that the Ostrowski-Reich theorem guarantees for SPD matrices and 0 < omega < 2."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from synth import CSR


def _random_dominant(n, seed):
    rng = np.random.default_rng(seed)
    d = np.where(rng.uniform(size=(n, n)) < 0.12, rng.uniform(-1, 1, (n, n)), 0.0)
    np.fill_diagonal(d, 0.0)
    np.fill_diagonal(d, np.abs(d).sum(axis=1) + rng.uniform(0.5, 1.5, n))
    m = sp.csr_matrix(d)
    m.sort_indices()
    return d, CSR(n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())


@pytest.mark.parametrize("omega", [0.7, 1.0, 1.4])
@pytest.mark.parametrize("symmetric", [False, True])
def test_sweep_equals_its_matrix_form(omega, symmetric):
    # forward: (D/omega + L) x1 = b - (U + (1 - 1/omega) D) x0; backward swaps L and U
    d, A = _random_dominant(40, 3)
    D = np.diag(np.diag(d))
    L, U = np.tril(d, -1), np.triu(d, 1)
    b = synth.rhs(40, 2, 4)
    x0 = synth.rhs(40, 2, 5)
    x1 = np.linalg.solve(D / omega + L, b - (U + (1 - 1 / omega) * D) @ x0)
    if symmetric:
        x1 = np.linalg.solve(D / omega + U, b - (L + (1 - 1 / omega) * D) @ x1)
    got = oracle.sor(A, b, x0, omega=omega, sweeps=1, symmetric=symmetric)
    assert np.linalg.norm(got - x1) <= 1e-13 * np.linalg.norm(x1)


def test_gauss_seidel_solves_a_lower_triangle_in_one_sweep():
    T = synth.random_lower(300, 0.02, 6)
    b = synth.rhs(300, 1, 7)[:, 0]
    ref = spla.spsolve_triangular(T.to_scipy(), b, lower=True)
    got = oracle.sor(T, b, np.full(300, 5.0), omega=1.0, sweeps=1)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("omega", [0.5, 1.0, 1.6])
def test_energy_norm_error_decreases_for_spd(omega):
    A = synth.diffusion2d(12, 11, 1.0, seed=8)
    Ad = A.to_dense()
    b = synth.rhs(A.n, 1, 9)[:, 0]
    xs = np.linalg.solve(Ad, b)
    x = np.zeros(A.n)
    prev = np.inf
    for _ in range(30):
        x = oracle.sor(A, b, x, omega=omega, sweeps=1, symmetric=True)
        e = x - xs
        cur = float(np.sqrt(e @ Ad @ e))
        assert cur < prev
        prev = cur
    assert prev < 0.5 * np.sqrt(xs @ Ad @ xs)


def test_zero_sweeps_and_errors():
    A = synth.poisson2d(4)
    b = synth.rhs(16, 1, 1)
    x0 = synth.rhs(16, 1, 2)
    assert np.array_equal(oracle.sor(A, b, x0, sweeps=0), x0)
    v = A.val.copy()
    v[A.col == np.repeat(np.arange(16), np.diff(A.rowptr))] = 0.0
    with pytest.raises(oracle.OracleError):
        oracle.sor(CSR(16, A.rowptr, A.col, v), b, x0)
