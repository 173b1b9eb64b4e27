"""Pins of the oracle's level analysis (eq. (2)), level map (eq. (3)) and
reordering (Algorithm 1) against brute force, grid closed forms and the
invariants the paper states."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
import synth
from synth import CSR


def _longest_path_levels(T: CSR, upper: bool):
    """eq. (2) evaluated by recursion over rows in dependency order."""
    n = T.n
    lev = [0] * n
    order = range(n - 1, -1, -1) if upper else range(n)
    for i in order:
        m = 0
        for p in range(T.rowptr[i], T.rowptr[i + 1]):
            j = int(T.col[p])
            if j != i:
                m = max(m, lev[j])
        lev[i] = 1 + m
    return np.array(lev, dtype=np.int32)


def _transpose(T):
    m = T.to_scipy().T.tocsr()
    m.sort_indices()
    return CSR(T.n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())


@settings(max_examples=40, deadline=None)
@given(n=st.integers(1, 120), dens=st.floats(0.0, 0.2), seed=st.integers(0, 10**6),
       dense_row=st.booleans())
def test_kahn_equals_longest_path(n, dens, seed, dense_row):
    L = synth.random_lower(n, dens, seed, dense_row=(n // 2 if dense_row and n > 2 else None))
    lev, nlev = oracle.levels(L)
    ref = _longest_path_levels(L, upper=False)
    assert np.array_equal(lev, ref)
    assert nlev == (ref.max() if n else 0)
    U = _transpose(L)
    levu, nlevu = oracle.levels(U, upper=True)
    assert np.array_equal(levu, _longest_path_levels(U, upper=True))


def test_special_cases():
    n = 64
    D = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    lev, nlev = oracle.levels(D)
    assert nlev == 1 and np.all(lev == 1)
    # lower bidiagonal: n levels of one row each
    rp = np.concatenate([[0], np.arange(1, 2 * n, 2)]).astype(np.int32)
    ci = np.concatenate([[0]] + [[i - 1, i] for i in range(1, n)]).astype(np.int32)
    B = CSR(n, rp, ci, np.ones(ci.shape[0]))
    lev, nlev = oracle.levels(B)
    assert nlev == n and np.array_equal(lev, np.arange(1, n + 1))


@pytest.mark.parametrize("nx,ny", [(64, 64), (7, 13), (1, 9)])
def test_2d_ilu0_level_closed_form(nx, ny):
    L, U = oracle.ilu0(synth.poisson2d(nx, ny))
    lev, nlev = oracle.levels(L)
    x = np.tile(np.arange(nx), ny)
    y = np.repeat(np.arange(ny), nx)
    assert np.array_equal(lev, x + y + 1)
    assert nlev == nx + ny - 1
    levu, nlevu = oracle.levels(U, upper=True)
    assert np.array_equal(levu, (nx - 1 - x) + (ny - 1 - y) + 1)
    assert nlevu == nlev


def test_3d_ilu0_level_closed_form():
    s = 12
    L, U = oracle.ilu0(synth.poisson3d(s))
    lev, nlev = oracle.levels(L)
    g = np.indices((s, s, s))  # z, y, x
    ref = (g[2] + g[1] + g[0]).ravel() + 1
    assert np.array_equal(lev, ref)
    assert nlev == 3 * s - 2


@pytest.mark.slow
def test_128cube_level_sizes():
    # 3D 7-point ILU(0) on 128^3: 382 levels; level k holds #{x+y+z = k-1}
    # rows, maximum 12,288 (k = 191, 192) and mean 2^21 / 382
    A = synth.poisson3d(128)
    L, _ = oracle.ilu0(A)
    lev, nlev = oracle.levels(L)
    assert nlev == 382
    sizes = np.bincount(lev)[1:]
    assert sizes.max() == 12288
    assert sizes.sum() == 128 ** 3
    # closed form for the level sizes: coefficients of (1 + t + ... + t^127)^3
    c = np.ones(128, dtype=np.int64)
    ref = np.convolve(np.convolve(c, c), c)
    assert np.array_equal(sizes, ref)


@pytest.mark.parametrize("s", [5, 9])
def test_iluk1_level_closed_forms(s):
    L, U = oracle.iluk(synth.poisson2d(s), 1)
    lev, nlev = oracle.levels(L)
    x = np.tile(np.arange(s), s)
    y = np.repeat(np.arange(s), s)
    assert np.array_equal(lev, x + 2 * y + 1)
    assert nlev == 3 * s - 2
    L3, _ = oracle.iluk(synth.poisson3d(s), 1)
    lev3, nlev3 = oracle.levels(L3)
    g = np.indices((s, s, s))
    assert np.array_equal(lev3, (g[2] + 2 * g[1] + 3 * g[0]).ravel() + 1)
    assert nlev3 == 6 * s - 5


def _brute_perm(level, upper):
    n = len(level)
    idx = list(range(n))
    key = [(int(level[i]), (n - 1 - i) if upper else i) for i in idx]
    return np.array(sorted(idx, key=lambda i: key[i]), dtype=np.int32)


@pytest.mark.parametrize("upper", [False, True])
@pytest.mark.parametrize("seed", range(5))
def test_level_map_brute_force(seed, upper):
    L = synth.random_lower(300, 0.02, seed)
    T = _transpose(L) if upper else L
    lev, nlev = oracle.levels(T, upper=upper)
    levelptr, perm, iperm = oracle.level_schedule(lev, nlev, upper=upper)
    assert np.array_equal(perm, _brute_perm(lev, upper))
    assert np.array_equal(iperm[perm], np.arange(T.n))
    # levelptr[k] = number of rows of level <= k
    for k in range(nlev + 1):
        assert levelptr[k] == np.count_nonzero(lev <= k)
    # sets S_k: consecutive, sorted by the problem's index
    for k in range(nlev):
        seg = perm[levelptr[k]:levelptr[k + 1]]
        assert np.all(lev[seg] == k + 1)
        assert np.all(np.diff(seg) < 0) if upper else np.all(np.diff(seg) > 0)


@pytest.mark.parametrize("upper", [False, True])
def test_reorder_is_still_triangular_and_similar(upper):
    L = synth.random_lower(150, 0.05, seed=3)
    T = _transpose(L) if upper else L
    lev, nlev = oracle.levels(T, upper=upper)
    _, perm, iperm = oracle.level_schedule(lev, nlev, upper=upper)
    Tp = oracle.reorder(T, perm, iperm)
    # L' is lower triangular in the new numbering; diagonal last per row
    for r in range(Tp.n):
        c = Tp.col[Tp.rowptr[r]:Tp.rowptr[r + 1]]
        assert np.all(c[:-1] < r) and c[-1] == r
    # L'_{m(i) m(j)} = T_ij
    P = np.zeros((T.n, T.n))
    P[np.arange(T.n), perm] = 1.0
    assert np.array_equal(Tp.to_dense(), P @ T.to_dense() @ P.T)


def test_hec_roundtrip_helper():
    # a hand-made HEC of a 3x3 lower matrix, ELL width 1 (column-major, ld 4)
    n, w, ld = 3, 1, 4
    ell_col = np.array([3, 0, 1, 3])  # row 0 padded (col n), rows 1, 2 one entry
    ell_val = np.array([0.0, -1.0, -2.0, 0.0])
    csr_ptr = np.array([0, 1, 2, 4])
    csr_col = np.array([0, 1, 0, 2])
    csr_val = np.array([1.0, 1.0, 5.0, 1.0])
    T = oracle.hec_to_csr(n, w, ld, ell_col, ell_val, csr_ptr, csr_col, csr_val)
    ref = np.array([[1.0, 0, 0], [-1.0, 1.0, 0], [5.0, -2.0, 1.0]])
    assert np.array_equal(T.to_dense(), ref)
    assert list(T.col[T.rowptr[2]:T.rowptr[3]]) == [1, 0, 2]
