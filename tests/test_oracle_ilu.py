"""Pins of the oracle's incomplete factorizations (Section 3): pattern
identities, closed recurrences, exact-LU limits and fill-pattern forms."""
import numpy as np
import pytest

import oracle
import synth


def _dense_nopivot_lu(d):
    """Doolittle LU without pivoting (textbook definition)."""
    n = d.shape[0]
    L = np.eye(n)
    U = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            U[i, j] = d[i, j] - L[i, :i] @ U[:i, j]
        for j in range(i + 1, n):
            L[j, i] = (d[j, i] - L[j, :i] @ U[:i, i]) / U[i, i]
    return L, U


@pytest.mark.parametrize("gen", [lambda: synth.poisson2d(9, 7), lambda: synth.poisson3d(6),
                                 lambda: synth.diffusion3d(6, 5, 4, 2.0, 3)])
def test_ilu0_matches_a_on_its_pattern(gen):
    A = gen()
    L, U = oracle.ilu0(A)
    Ad = A.to_dense()
    LU = L.to_dense() @ U.to_dense()
    mask = Ad != 0
    scale = np.abs(Ad).max()
    assert np.abs(LU[mask] - Ad[mask]).max() <= 1e-13 * scale
    # factors keep A's pattern exactly
    assert np.array_equal((np.tril(Ad, -1) != 0), (np.tril(L.to_dense(), -1) != 0))
    assert np.array_equal((np.triu(Ad) != 0), (U.to_dense() != 0))
    # L rows end with an explicit unit diagonal; U rows start with the diagonal
    for i in range(A.n):
        assert L.col[L.rowptr[i + 1] - 1] == i and L.val[L.rowptr[i + 1] - 1] == 1.0
        assert U.col[U.rowptr[i]] == i


def test_ilu0_5point_recurrence():
    # u(x,y) = 4 - 1/u(x-1,y) - 1/u(x,y-1); l to a neighbour = -1/u(neighbour)
    nx, ny = 11, 8
    L, U = oracle.ilu0(synth.poisson2d(nx, ny))
    u = np.zeros((ny, nx))
    for y in range(ny):
        for x in range(nx):
            v = 4.0
            if x > 0:
                v -= 1.0 / u[y, x - 1]
            if y > 0:
                v -= 1.0 / u[y - 1, x]
            u[y, x] = v
    assert np.allclose(np.diag(U.to_dense()), u.ravel(), rtol=1e-15, atol=0)
    Ld = L.to_dense()
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            if x > 0:
                assert np.isclose(Ld[i, i - 1], -1.0 / u[y, x - 1], rtol=1e-15)
            if y > 0:
                assert np.isclose(Ld[i, i - nx], -1.0 / u[y - 1, x], rtol=1e-15)


@pytest.mark.parametrize("kind", ["iluk", "ilut"])
def test_full_fill_is_the_exact_lu(kind):
    A = synth.diffusion2d(5, 4, 1.0, seed=2)
    if kind == "iluk":
        L, U = oracle.iluk(A, A.n)
    else:
        L, U = oracle.ilut(A, A.n, 0.0)
    Lr, Ur = _dense_nopivot_lu(A.to_dense())
    assert np.allclose(L.to_dense(), Lr, rtol=1e-12, atol=1e-14)
    assert np.allclose(U.to_dense(), Ur, rtol=1e-12, atol=1e-14)


def test_iluk0_equals_ilu0():
    A = synth.diffusion3d(5, 6, 4, 1.5, seed=4)
    L0, U0 = oracle.ilu0(A)
    Lk, Uk = oracle.iluk(A, 0)
    for a, b in ((L0, Lk), (U0, Uk)):
        assert np.array_equal(a.rowptr, b.rowptr)
        assert np.array_equal(a.col, b.col)
        assert np.array_equal(a.val, b.val)


def test_iluk1_fill_pattern_closed_forms():
    s = 8
    L, _ = oracle.iluk(synth.poisson2d(s), 1)
    i = s * (s // 2) + s // 2  # an interior row
    offs = sorted(i - L.col[L.rowptr[i]:L.rowptr[i + 1] - 1])
    assert offs == sorted([1, s - 1, s])
    L3, _ = oracle.iluk(synth.poisson3d(s), 1)
    i = s * s * (s // 2) + s * (s // 2) + s // 2
    offs = sorted(i - L3.col[L3.rowptr[i]:L3.rowptr[i + 1] - 1])
    assert offs == sorted([1, s - 1, s, s * s - s, s * s - 1, s * s])


def test_ilut_limits_and_invariants():
    A = synth.diffusion3d(6, 6, 6, 2.0, seed=5)
    # p = 0: L = I, U = diag(A)
    L, U = oracle.ilut(A, 0, 1e-3)
    assert np.array_equal(L.to_dense(), np.eye(A.n))
    assert np.array_equal(U.to_dense(), np.diag(np.diag(A.to_dense())))
    # general case: at most p per part, sorted rows, diagonal kept
    p, tau = 3, 1e-3
    L, U = oracle.ilut(A, p, tau)
    for r in range(A.n):
        lc = L.col[L.rowptr[r]:L.rowptr[r + 1]]
        uc = U.col[U.rowptr[r]:U.rowptr[r + 1]]
        assert len(lc) - 1 <= p and len(uc) - 1 <= p
        assert lc[-1] == r and uc[0] == r
        assert np.all(np.diff(lc) > 0) and np.all(np.diff(uc) > 0)
    # a large tau keeps only the diagonal-related part
    L2, U2 = oracle.ilut(A, 10, 10.0)
    assert L2.nnz == A.n and U2.nnz == A.n


def test_example1_sizes_golden():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "example1_sizes.txt")
    vals = dict(line.split() for line in open(path) if line.strip() and not line.startswith("#"))
    A = synth.poisson3d(100)
    assert A.n == int(vals["n"]) and A.nnz == int(vals["nnz"])
