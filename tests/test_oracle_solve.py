"""Pins of the oracle's triangular solves (eq. (1)) against closed forms,
library routines on small inputs and the backward-error bound."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from synth import CSR


def _csr_from_dense(d):
    m = sp.csr_matrix(d)
    m.sort_indices()
    return CSR(d.shape[0], m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))


def _bidiag(n, a, upper=False):
    d = np.eye(n)
    for i in range(1, n):
        if upper:
            d[i - 1, i] = -a
        else:
            d[i, i - 1] = -a
    return _csr_from_dense(d)


def test_identity_is_exact():
    n = 50
    L = _csr_from_dense(np.eye(n))
    b = synth.rhs(n, 3, 11)
    assert np.array_equal(oracle.lower_solve(L, b), b)
    assert np.array_equal(oracle.upper_solve(L, b), b)


def test_diagonal_is_exact_division():
    n = 40
    d = np.random.default_rng(1).uniform(0.5, 3.0, n)
    D = _csr_from_dense(np.diag(d))
    b = synth.rhs(n, 1, 12)[:, 0]
    assert np.array_equal(oracle.lower_solve(D, b), b / d)
    assert np.array_equal(oracle.upper_solve(D, b), b / d)


def test_unit_bidiagonal_closed_forms():
    n = 1000
    # L: 1 on the diagonal, -1 below; b = 1 gives x_i = i (1-based), exactly
    x = oracle.lower_solve(_bidiag(n, 1.0), np.ones(n))
    assert np.array_equal(x, np.arange(1, n + 1, dtype=float))
    # its upper mirror gives x_i = n - i + 1
    x = oracle.upper_solve(_bidiag(n, 1.0, upper=True), np.ones(n))
    assert np.array_equal(x, np.arange(n, 0, -1, dtype=float))
    # subdiagonal -a with b = e_1 gives x_i = a^(i-1); a = 1/2 is exact
    e1 = np.zeros(n)
    e1[0] = 1.0
    x = oracle.lower_solve(_bidiag(60, 0.5), e1[:60])
    assert np.array_equal(x, 0.5 ** np.arange(60))


def test_unit_flag_skips_the_diagonal():
    n = 30
    d = np.tril(np.random.default_rng(2).uniform(-1, 1, (n, n)), -1) / n + np.diag(np.full(n, 3.0))
    L = _csr_from_dense(d)
    b = synth.rhs(n, 1, 3)[:, 0]
    xu = oracle.lower_solve(L, b, unit=True)
    ref = sla.solve_triangular(np.tril(d, -1) + np.eye(n), b, lower=True, unit_diagonal=True)
    assert np.allclose(xu, ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n", [1, 2, 17, 64])
def test_dense_library_case(seed, n):
    rng = np.random.default_rng(seed)
    mask = rng.uniform(size=(n, n)) < 0.4
    d = np.where(mask, rng.uniform(-1, 1, (n, n)), 0.0)
    lo = np.tril(d, -1) / max(1, n) * 4 + np.diag(rng.uniform(1, 2, n))
    up = np.triu(d, 1) / max(1, n) * 4 + np.diag(rng.uniform(1, 2, n))
    b = rng.uniform(-1, 1, (n, 2))
    xl = oracle.lower_solve(_csr_from_dense(lo), b)
    xu = oracle.upper_solve(_csr_from_dense(up), b)
    assert np.allclose(xl, sla.solve_triangular(lo, b, lower=True), rtol=1e-13, atol=1e-14)
    assert np.allclose(xu, sla.solve_triangular(up, b, lower=False), rtol=1e-13, atol=1e-14)


def test_sparse_library_case_and_backward_error():
    L = synth.random_lower(3000, 0.002, seed=4)
    b = synth.rhs(L.n, 1, 5)[:, 0]
    x = oracle.lower_solve(L, b)
    ref = spla.spsolve_triangular(L.to_scipy(), b, lower=True)
    assert np.allclose(x, ref, rtol=1e-12, atol=1e-13)
    # componentwise backward error: |L x - b| <= c n eps |L| |x|
    S = L.to_scipy()
    res = np.abs(S @ x - b)
    bound = 4 * L.n * np.finfo(float).eps * (abs(S) @ np.abs(x))
    assert np.all(res <= bound + 1e-300)


def test_multi_rhs_equals_columnwise():
    L = synth.random_lower(500, 0.01, seed=6)
    U = CSR(L.n, *_transpose(L))
    b = synth.rhs(L.n, 4, 7)
    x = oracle.lower_solve(L, b)
    xu = oracle.upper_solve(U, b)
    for r in range(4):
        assert np.array_equal(x[:, r], oracle.lower_solve(L, b[:, r]))
        assert np.array_equal(xu[:, r], oracle.upper_solve(U, b[:, r]))


def _transpose(T):
    m = T.to_scipy().T.tocsr()
    m.sort_indices()
    return m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy()


def test_tridiagonal_ilu0_is_exact_lu():
    # T = tridiag(-1, 2, -1): ILU(0) equals the exact LU with
    # u_ii = (i+1)/i and l_{i,i-1} = -(i-1)/i (1-based)
    n = 200
    d = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    A = _csr_from_dense(d)
    L, U = oracle.ilu0(A)
    i = np.arange(1, n + 1, dtype=float)
    udiag = np.diag(U.to_dense())
    assert np.allclose(udiag, (i + 1) / i, rtol=1e-14)
    lsub = np.diag(L.to_dense(), -1)
    assert np.allclose(lsub, -(i[1:] - 1) / i[1:], rtol=1e-14)
    xt = np.random.default_rng(8).uniform(-1, 1, n)
    z = oracle.ilu_apply(L, U, d @ xt)
    assert np.allclose(z, xt, rtol=1e-11, atol=1e-12)


def test_single_precision_solves():
    n = 2000
    x = oracle.lower_solve_f32(CSR(n, *_bidiag_arrays(n)), np.ones(n, np.float32), unit=False)
    assert x.dtype == np.float32
    assert np.array_equal(x, np.arange(1, n + 1, dtype=np.float32))
    L = synth.random_lower(800, 0.01, seed=9)
    b = synth.rhs(L.n, 1, 10)[:, 0]
    x64 = oracle.lower_solve(L, b)
    x32 = oracle.lower_solve_f32(oracle.to_f32(L), b)
    err = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    assert err < 1e-5
    assert err > 0  # it really ran in single precision


def _bidiag_arrays(n):
    m = _bidiag(n, 1.0)
    return m.rowptr, m.col, m.val


def test_errors_are_reported():
    bad = _csr_from_dense(np.array([[1.0, 2.0], [0.0, 1.0]]))
    with pytest.raises(oracle.OracleError):
        oracle.lower_solve(bad, np.ones(2))
    nodiag = _csr_from_dense(np.array([[1.0, 0.0], [1.0, 0.0]]))
    with pytest.raises(oracle.OracleError):
        oracle.lower_solve(nodiag, np.ones(2))
    # with a unit diagonal the missing entry is fine
    assert np.array_equal(oracle.lower_solve(nodiag, np.ones(2), unit=True), np.array([1.0, 0.0]))


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("upper,unit", [(False, False), (False, True), (True, False)])
def test_omp_level_solve_equals_serial_substitution(threads, upper, unit):
    # the multithreaded CPU baseline does the serial per-row arithmetic in
    # level order (Algorithm 2 on the host), so it must agree bit for bit
    T = synth.random_lower(700, 0.01, 21, unit=unit, dense_row=350)
    if upper:
        T = CSR(T.n, *_transpose(T))
    b = synth.rhs(T.n, 3, 22)
    ref = oracle.upper_solve(T, b, unit=unit) if upper else oracle.lower_solve(T, b, unit=unit)
    got = oracle.LevelSolveCPU(T, upper=upper, unit=unit).solve(b, threads=threads)
    assert np.array_equal(got, ref)


def test_omp_level_solve_on_ilu0_factors():
    A = synth.poisson3d(12, 10, 9)
    L, U = oracle.ilu0(A)
    r = synth.rhs(A.n, 1, 2)
    sl, su = oracle.LevelSolveCPU(L, unit=True), oracle.LevelSolveCPU(U, upper=True)
    assert sl.nlev == 12 + 10 + 9 - 2 and su.nlev == sl.nlev
    assert np.array_equal(su.solve(sl.solve(r)), oracle.ilu_apply(L, U, r))
    assert oracle.omp_threads() >= 1
