"""CPU oracle for the level-scheduled triangular-solve path.

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or calls
anything here; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the GPU path: its arithmetic is
plain C (``orc.c``, double precision, no FMA contraction) and NumPy, and it
takes its inputs from the seeded generators in ``synth`` (which hold none of
the method's arithmetic).

Each function names the passage of the paper (Chen, Liu and Yang, "Parallel
Triangular Solvers on GPU") it follows.  Functions with no independent pin
say so in their docstring ("parity unpinned").
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from synth import CSR

from . import build as _build

_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)
_F32P = ctypes.POINTER(ctypes.c_float)
_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = _bind(ctypes.CDLL(_build.build()))
    return _lib


def use_native_build(dest_dir: str) -> str:
    """Switch this process to a -O3 -march=native build of the oracle made
    for the current host in dest_dir (the benchmark's CPU baseline); the
    arithmetic is unchanged (no contraction, no reassociation).  Returns the
    library path."""
    global _lib
    path = _build.build_native(dest_dir)
    _lib = _bind(ctypes.CDLL(path))
    return path


def _bind(lib):
    if True:
        i32, vp = ctypes.c_int32, ctypes.c_void_p
        for name in ("orc_lower_solve", "orc_upper_solve", "orc_lower_solve_f32",
                     "orc_upper_solve_f32"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [i32, vp, vp, vp, ctypes.c_int, i32, vp, vp]
        lib.orc_levels_kahn.restype = ctypes.c_int
        lib.orc_levels_kahn.argtypes = [i32, vp, vp, ctypes.c_int, vp, vp]
        lib.orc_spmv.restype = None
        lib.orc_spmv.argtypes = [i32, vp, vp, vp, i32, vp, vp]
        lib.orc_ilu0.restype = ctypes.c_int
        lib.orc_ilu0.argtypes = [i32, vp, vp, vp, vp]
        lib.orc_iluk.restype = ctypes.c_int
        lib.orc_iluk.argtypes = [i32, vp, vp, vp, i32, ctypes.POINTER(_I32P),
                                 ctypes.POINTER(_I32P), ctypes.POINTER(_F64P)]
        lib.orc_ilut.restype = ctypes.c_int
        lib.orc_ilut.argtypes = [i32, vp, vp, vp, i32, ctypes.c_double,
                                 ctypes.POINTER(_I32P), ctypes.POINTER(_I32P), ctypes.POINTER(_F64P),
                                 ctypes.POINTER(_I32P), ctypes.POINTER(_I32P), ctypes.POINTER(_F64P)]
        lib.orc_sor.restype = ctypes.c_int
        lib.orc_sor.argtypes = [i32, vp, vp, vp, ctypes.c_double, i32, vp, vp, i32, ctypes.c_int]
        lib.orc_free.restype = None
        lib.orc_free.argtypes = [vp]
    return lib


class OracleError(RuntimeError):
    pass


_RC = {-1: "entry on the wrong side of the diagonal", -2: "missing diagonal",
       -3: "zero pivot", -4: "allocation failure", -5: "bad argument"}


def _check(rc):
    if rc != 0:
        raise OracleError(_RC.get(rc, "error %d" % rc))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_args(T: CSR):
    rp = np.ascontiguousarray(T.rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(T.col, dtype=np.int32)
    return rp, ci


def _as2d(b):
    b = np.asarray(b)
    return (b[:, None], True) if b.ndim == 1 else (b, False)


# --------------------------------------------------------------------------
# Triangular solves: eq. (1), plain substitution in natural order.
# --------------------------------------------------------------------------

def lower_solve(L: CSR, b, unit: bool = False) -> np.ndarray:
    """Solve L x = b by forward substitution (eq. (1), first half)."""
    b2, flat = _as2d(b)
    b2 = np.ascontiguousarray(b2, dtype=np.float64)
    x = np.empty_like(b2)
    rp, ci = _csr_args(L)
    v = np.ascontiguousarray(L.val, dtype=np.float64)
    _check(_L().orc_lower_solve(L.n, _p(rp), _p(ci), _p(v), int(unit), b2.shape[1], _p(b2), _p(x)))
    return x[:, 0] if flat else x


def upper_solve(U: CSR, b, unit: bool = False) -> np.ndarray:
    """Solve U x = b by backward substitution (eq. (1), second half)."""
    b2, flat = _as2d(b)
    b2 = np.ascontiguousarray(b2, dtype=np.float64)
    x = np.empty_like(b2)
    rp, ci = _csr_args(U)
    v = np.ascontiguousarray(U.val, dtype=np.float64)
    _check(_L().orc_upper_solve(U.n, _p(rp), _p(ci), _p(v), int(unit), b2.shape[1], _p(b2), _p(x)))
    return x[:, 0] if flat else x


def lower_solve_f32(L: CSR, b, unit: bool = False) -> np.ndarray:
    """Forward substitution in single precision (factors, vectors and sums)."""
    b2, flat = _as2d(b)
    b2 = np.ascontiguousarray(b2, dtype=np.float32)
    x = np.empty_like(b2)
    rp, ci = _csr_args(L)
    v = np.ascontiguousarray(L.val, dtype=np.float32)
    _check(_L().orc_lower_solve_f32(L.n, _p(rp), _p(ci), _p(v), int(unit), b2.shape[1], _p(b2), _p(x)))
    return x[:, 0] if flat else x


def upper_solve_f32(U: CSR, b, unit: bool = False) -> np.ndarray:
    """Backward substitution in single precision (factors, vectors and sums)."""
    b2, flat = _as2d(b)
    b2 = np.ascontiguousarray(b2, dtype=np.float32)
    x = np.empty_like(b2)
    rp, ci = _csr_args(U)
    v = np.ascontiguousarray(U.val, dtype=np.float32)
    _check(_L().orc_upper_solve_f32(U.n, _p(rp), _p(ci), _p(v), int(unit), b2.shape[1], _p(b2), _p(x)))
    return x[:, 0] if flat else x


def sor(A: CSR, b, x0, omega: float = 1.0, sweeps: int = 1, symmetric: bool = False) -> np.ndarray:
    """SOR sweeps in the elementwise textbook form (Gauss-Seidel for
    omega = 1; the smoothers Section 1 names): row by row, in place,
    x_i <- (1 - omega) x_i + omega (b_i - sum_{j != i} a_ij x_j) / a_ii;
    forward rows 0..n-1, then (symmetric) rows n-1..0.  Returns the new x."""
    b2, flat = _as2d(b)
    b2 = np.ascontiguousarray(b2, dtype=np.float64)
    x = np.ascontiguousarray(np.array(_as2d(x0)[0], dtype=np.float64))
    rp, ci = _csr_args(A)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    _check(_L().orc_sor(A.n, _p(rp), _p(ci), _p(v), float(omega), b2.shape[1], _p(b2), _p(x), int(sweeps),
                        int(bool(symmetric))))
    return x[:, 0] if flat else x


def spmv(A: CSR, x) -> np.ndarray:
    """y = A x in natural entry order (support for residuals b - A x)."""
    x2, flat = _as2d(x)
    x2 = np.ascontiguousarray(x2, dtype=np.float64)
    y = np.empty_like(x2)
    rp, ci = _csr_args(A)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    _L().orc_spmv(A.n, _p(rp), _p(ci), _p(v), x2.shape[1], _p(x2), _p(y))
    return y[:, 0] if flat else y


# --------------------------------------------------------------------------
# Preprocessing, Algorithm 1: levels (eq. (2)), map (eq. (3)), reorder, HEC.
# --------------------------------------------------------------------------

def levels(T: CSR, upper: bool = False):
    """Level of every unknown, eq. (2), by Kahn peeling of the dependency DAG.

    Only off-diagonal stored entries count (structural, explicit zeros
    included); levels are 1-based and a row with no dependency has level 1.
    For an upper triangle the dependencies point to larger indices, which is
    eq. (2) applied to the problem reversed by t(i) = n-1-i.
    Returns (level int32[n], nlev).
    """
    rp, ci = _csr_args(T)
    lev = np.empty(T.n, dtype=np.int32)
    nlev = ctypes.c_int32(0)
    _check(_L().orc_levels_kahn(T.n, _p(rp), _p(ci), int(upper), _p(lev), ctypes.addressof(nlev)))
    return lev, int(nlev.value)


def level_schedule(level: np.ndarray, nlev: int, upper: bool = False):
    """Level sets S_k and the map m of eq. (3).

    ``levelptr[k]`` is the first position of level k+1 (sum of N_j, j <= k);
    ``perm[r]`` is the original row at new position r (level 1 first; inside
    a level ascending index of the problem solved, i.e. descending original
    index for an upper triangle after the reversal t); ``iperm = m`` maps
    original rows to new positions.
    """
    n = level.shape[0]
    counts = np.bincount(level, minlength=nlev + 1)[1:]
    levelptr = np.zeros(nlev + 1, dtype=np.int64)
    np.cumsum(counts, out=levelptr[1:])
    problem_index = np.arange(n)[::-1] if upper else np.arange(n)
    key = level[problem_index]
    perm = problem_index[np.argsort(key, kind="stable")]
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)
    return levelptr.astype(np.int32), perm.astype(np.int32), iperm.astype(np.int32)


def reorder(T: CSR, perm: np.ndarray, iperm: np.ndarray) -> CSR:
    """L' with L'_{m(i) m(j)} = T_ij (Algorithm 1, step 3).

    Row r of L' is original row perm[r]; its off-diagonal entries keep their
    original (ascending original column) order and the diagonal, if stored,
    is moved to the end of the row.  The result is lower triangular in the
    new numbering for a lower triangle, and for an upper triangle ordered by
    its reversed levels.
    """
    n = T.n
    rp, ci, v = T.rowptr, T.col, T.val
    rows, cols, vals = [], [], []
    newptr = np.zeros(n + 1, dtype=np.int64)
    for r in range(n):
        i = int(perm[r])
        seg = slice(int(rp[i]), int(rp[i + 1]))
        c, x = ci[seg], v[seg]
        off = c != i
        cc = np.concatenate([iperm[c[off]], iperm[c[~off]]])
        xx = np.concatenate([x[off], x[~off]])
        cols.append(cc)
        vals.append(xx)
        newptr[r + 1] = newptr[r] + cc.shape[0]
    return CSR(n, newptr.astype(np.int32),
               np.concatenate(cols).astype(np.int32) if cols else np.empty(0, np.int32),
               np.concatenate(vals) if vals else np.empty(0, v.dtype))


def hec_to_csr(n: int, width: int, ld: int, ell_col, ell_val, csr_ptr, csr_col, csr_val,
               pad_col: int | None = None) -> CSR:
    """Rebuild CSR from an HEC matrix (Section 2.1): row r is its ELL slots
    e = 0..width-1 at ``e*ld + r`` (column-major) that are not padding, then
    its CSR-remainder entries.  Used to check the HEC round trip exactly."""
    pad_col = n if pad_col is None else pad_col
    ell_col = np.asarray(ell_col).reshape(width, ld) if width else np.zeros((0, ld), np.int32)
    ell_val = np.asarray(ell_val).reshape(width, ld) if width else np.zeros((0, ld))
    csr_ptr = np.asarray(csr_ptr)
    rows_c, rows_v, ptr = [], [], np.zeros(n + 1, dtype=np.int64)
    for r in range(n):
        ec = ell_col[:, r]
        keep = ec != pad_col
        c = np.concatenate([ec[keep], np.asarray(csr_col)[csr_ptr[r]:csr_ptr[r + 1]]])
        x = np.concatenate([ell_val[:, r][keep], np.asarray(csr_val)[csr_ptr[r]:csr_ptr[r + 1]]])
        rows_c.append(c)
        rows_v.append(x)
        ptr[r + 1] = ptr[r] + c.shape[0]
    return CSR(n, ptr.astype(np.int32), np.concatenate(rows_c).astype(np.int32),
               np.concatenate(rows_v))


# --------------------------------------------------------------------------
# Incomplete factorizations, Section 3.
# --------------------------------------------------------------------------

def _split_lu(n, rp, ci, lu):
    """Split a combined factor into L (strict part + explicit unit diagonal,
    diagonal last in each row) and U (diagonal first)."""
    rows = np.repeat(np.arange(n), np.diff(rp))
    lower = ci < rows
    upper = ~lower
    lcount = np.bincount(rows[lower], minlength=n) + 1
    lrp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lcount, out=lrp[1:])
    lci = np.empty(int(lrp[-1]), dtype=np.int32)
    lv = np.empty(int(lrp[-1]))
    # rows are sorted, so a row's strict-lower entries lead it: entry p keeps
    # its offset p - rp[row]; the unit diagonal then closes the row
    p_idx = np.flatnonzero(lower)
    pos = lrp[rows[lower]] + (p_idx - np.asarray(rp)[rows[lower]])
    lci[pos] = ci[lower]
    lv[pos] = lu[lower]
    lci[lrp[1:] - 1] = np.arange(n)
    lv[lrp[1:] - 1] = 1.0
    ucount = np.bincount(rows[upper], minlength=n)
    urp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(ucount, out=urp[1:])
    L = CSR(n, lrp.astype(np.int32), lci, lv)
    U = CSR(n, urp.astype(np.int32), ci[upper].astype(np.int32), lu[upper].copy())
    return L, U


def ilu0(A: CSR):
    """ILU(0): IKJ elimination restricted to A's pattern (Section 3; Saad's
    textbook form).  Returns (L, U): L unit lower with the 1.0 diagonal stored
    last in each row, U upper with the diagonal first."""
    rp, ci = _csr_args(A)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    lu = np.empty_like(v)
    _check(_L().orc_ilu0(A.n, _p(rp), _p(ci), _p(v), _p(lu)))
    return _split_lu(A.n, rp, ci, lu)


def _take(ptr, count, ctype):
    arr = np.ctypeslib.as_array(ptr, shape=(count,)).copy() if count else np.empty(0, ctype)
    _L().orc_free(ctypes.cast(ptr, ctypes.c_void_p))
    return arr


def iluk(A: CSR, k: int):
    """ILU(k): level-of-fill symbolic phase (lev = 0 on A's pattern, fill
    level lev_ik + lev_kj + 1, keep lev <= k), then IKJ on that pattern
    (Section 3; Saad's textbook form).  Returns (L, U) as ``ilu0``."""
    rp, ci = _csr_args(A)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    orp, oci, ov = _I32P(), _I32P(), _F64P()
    rc = _L().orc_iluk(A.n, _p(rp), _p(ci), _p(v), int(k), ctypes.byref(orp), ctypes.byref(oci),
                       ctypes.byref(ov))
    _check(rc)
    frp = _take(orp, A.n + 1, np.int32)
    nnz = int(frp[-1])
    fci = _take(oci, nnz, np.int32)
    fv = _take(ov, nnz, np.float64)
    return _split_lu(A.n, frp, fci, fv)


def ilut(A: CSR, p: int, tau: float):
    """ILUT(p, tau) with dual dropping (Section 3; Saad's textbook form):
    drop by tau * ||a_i||_2, keep the p largest in each of L and U (ties to
    the smaller column), diagonal always kept.  Returns (L, U) as ``ilu0``.

    Pinned at its limits (tau = 0 with p >= n is the exact LU; p = 0 gives
    L = I, U = diag(A)) and between them by a 6x6 worked example derived by
    hand (tests/golden/ilut_6x6_p2_tau0125.txt) on which a multiplier
    dropped after its division, a fill entry dropped by the final test, the
    p-largest rule, the tie rule and the inclusive threshold each matter.
    """
    rp, ci = _csr_args(A)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    ptrs = [_I32P(), _I32P(), _F64P(), _I32P(), _I32P(), _F64P()]
    rc = _L().orc_ilut(A.n, _p(rp), _p(ci), _p(v), int(p), float(tau),
                       *[ctypes.byref(q) for q in ptrs])
    _check(rc)
    n = A.n
    lrp = _take(ptrs[0], n + 1, np.int32)
    lci = _take(ptrs[1], int(lrp[-1]), np.int32)
    lv = _take(ptrs[2], int(lrp[-1]), np.float64)
    urp = _take(ptrs[3], n + 1, np.int32)
    uci = _take(ptrs[4], int(urp[-1]), np.int32)
    uv = _take(ptrs[5], int(urp[-1]), np.float64)
    # append the unit diagonal to L rows
    cnt = np.diff(lrp) + 1
    nrp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=nrp[1:])
    nci = np.empty(int(nrp[-1]), dtype=np.int32)
    nv = np.empty(int(nrp[-1]))
    mask = np.ones(int(nrp[-1]), dtype=bool)
    mask[nrp[1:] - 1] = False
    nci[mask] = lci
    nv[mask] = lv
    nci[~mask] = np.arange(n)
    nv[~mask] = 1.0
    return CSR(n, nrp.astype(np.int32), nci, nv), CSR(n, urp, uci, uv)


def ilu_apply(L: CSR, U: CSR, r, unit_l: bool = True) -> np.ndarray:
    """z = (LU)^{-1} r: L y = r, then U z = y (eq. (1))."""
    return upper_solve(U, lower_solve(L, r, unit=unit_l))


def to_f32(T: CSR) -> CSR:
    """Factors rounded once to single precision."""
    return CSR(T.n, T.rowptr, T.col, T.val.astype(np.float32))


def ilu_apply_f32(L32: CSR, U32: CSR, r, unit_l: bool = True) -> np.ndarray:
    """Mixed-precision preconditioner: round r to FP32, solve with FP32
    factors and FP32 sums, widen z to FP64."""
    y = lower_solve_f32(L32, np.asarray(r, dtype=np.float32), unit=unit_l)
    return upper_solve_f32(U32, y).astype(np.float64)


# --------------------------------------------------------------------------
# Multithreaded level-scheduled CPU baseline (Algorithm 2 on the host cores).
# --------------------------------------------------------------------------

_omp_lib = None


def _Lomp():
    global _omp_lib
    if _omp_lib is None:
        lib = ctypes.CDLL(_build.build_omp())
        i32, vp = ctypes.c_int32, ctypes.c_void_p
        lib.orc_level_solve_omp.restype = ctypes.c_int
        lib.orc_level_solve_omp.argtypes = [i32, vp, vp, vp, ctypes.c_int, ctypes.c_int, i32, vp, vp,
                                            i32, vp, vp, i32]
        lib.orc_omp_threads.restype = ctypes.c_int
        lib.orc_omp_threads.argtypes = []
        _omp_lib = lib
    return _omp_lib


def omp_threads() -> int:
    """Threads the OpenMP baseline uses by default on this host."""
    return int(_Lomp().orc_omp_threads())


class LevelSolveCPU:
    """One triangle prepared for the multithreaded level-scheduled CPU solve:
    levels by eq. (2) and level sets by eq. (3) (this module's own analysis),
    then every level's rows in parallel with the serial substitution's
    per-row arithmetic, so the result equals :func:`lower_solve` /
    :func:`upper_solve` bit for bit.  A host comparison baseline, not an
    oracle of its own."""

    def __init__(self, T: CSR, upper: bool = False, unit: bool = False):
        lev, nlev = levels(T, upper=upper)
        levelptr, perm, _ = level_schedule(lev, nlev, upper=upper)
        self.n, self.upper, self.unit, self.nlev = T.n, bool(upper), bool(unit), nlev
        self.rp, self.ci = _csr_args(T)
        self.v = np.ascontiguousarray(T.val, dtype=np.float64)
        self.levelptr = np.ascontiguousarray(levelptr, dtype=np.int32)
        self.perm = np.ascontiguousarray(perm, dtype=np.int32)

    def solve(self, b, threads: int = 0) -> np.ndarray:
        b2, flat = _as2d(b)
        b2 = np.ascontiguousarray(b2, dtype=np.float64)
        x = np.empty_like(b2)
        _check(_Lomp().orc_level_solve_omp(self.n, _p(self.rp), _p(self.ci), _p(self.v), int(self.unit),
                                           int(self.upper), self.nlev, _p(self.levelptr), _p(self.perm),
                                           b2.shape[1], _p(b2), _p(x), int(threads)))
        return x[:, 0] if flat else x


# --------------------------------------------------------------------------
# Restricted Additive Schwarz, Section 3 and eq. (4).
# --------------------------------------------------------------------------

@dataclass
class RASDomain:
    ext: np.ndarray  # global rows of the extended subdomain, ascending
    owned_local: np.ndarray  # positions (in ext) of the rows this subdomain owns
    owned_global: np.ndarray
    L: CSR
    U: CSR


def _submatrix(A: CSR, rows: np.ndarray) -> CSR:
    S = A.to_scipy()[rows][:, rows].tocsr()
    S.sort_indices()
    return CSR(len(rows), S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy())


def ras_setup(A: CSR, owner: np.ndarray, nsub: int, overlap: int = 1, kind: str = "ilu0",
              k: int = 0, tau: float = 0.0, p: int = 0):
    """RAS setup: subdomain i owns the rows with owner == i; its extended set
    adds ``overlap`` rings of graph neighbours in A; A_i = A[ext_i, ext_i]
    (couplings to rows outside are dropped) is factored by ILU(0), or by
    ILU(k) / ILUT(p, tau) for the block forms of Section 3 (with overlap 0
    these are block ILU(k) and block ILUT: one block per subdomain, the
    couplings between blocks dropped)."""
    if kind not in ("ilu0", "iluk", "ilut"):
        raise ValueError("unknown ILU kind %r" % kind)
    S = A.to_scipy()
    out = []
    for s in range(nsub):
        owned = np.flatnonzero(owner == s)
        ext = owned
        for _ in range(overlap):
            nb = np.unique(S[ext].indices)
            ext = np.union1d(ext, nb)
        Ai = _submatrix(A, ext)
        if kind == "ilu0":
            L, U = ilu0(Ai)
        elif kind == "iluk":
            L, U = iluk(Ai, k)
        else:
            L, U = ilut(Ai, p, tau)
        out.append(RASDomain(ext, np.searchsorted(ext, owned), owned, L, U))
    return out


def ras_apply(doms, r) -> np.ndarray:
    """z = sum_i R_i^0' (L_i U_i)^{-1} R_i r (eq. (4) applied block by block):
    restrict r to each extended subdomain, solve with its factors and write
    back only the owned rows."""
    r2, flat = _as2d(r)
    z = np.zeros_like(r2, dtype=np.float64)
    for d in doms:
        zi = ilu_apply(d.L, d.U, r2[d.ext])
        z[d.owned_global] = zi[d.owned_local]
    return z[:, 0] if flat else z


def ras_apply_f32(doms32, r) -> np.ndarray:
    """RAS with FP32 local factors and solves; r and z in FP64."""
    r2, flat = _as2d(r)
    z = np.zeros_like(r2, dtype=np.float64)
    for d in doms32:
        zi = ilu_apply_f32(d.L, d.U, r2[d.ext])
        z[d.owned_global] = zi[d.owned_local]
    return z[:, 0] if flat else z


def ras_to_f32(doms):
    return [RASDomain(d.ext, d.owned_local, d.owned_global, to_f32(d.L), to_f32(d.U)) for d in doms]


# --------------------------------------------------------------------------
# Krylov solvers: restarted GMRES (the paper's linear solver, Section 4) in
# its flexible right-preconditioned form, and BiCGSTAB.  One RHS per call.
# --------------------------------------------------------------------------

@dataclass
class KrylovInfo:
    iters: int
    relres: float  # true ||b - A x|| / ||b||
    converged: bool
    precond_applies: int


def fgmres(A: CSR, b: np.ndarray, M, m: int = 30, rtol: float = 1e-10, maxit: int = 10000,
           x0=None):
    """Restarted flexible GMRES(m), right preconditioned, modified
    Gram-Schmidt, Givens rotations, x0 = 0 by default.  A cycle ends when the
    rotated residual estimate reaches rtol (or after m steps); the solver then
    stops only if the true residual ||b - A x|| / ||b|| <= rtol."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return np.zeros(n), KrylovInfo(0, 0.0, True, 0)
    it = 0
    applies = 0
    while True:
        r = b - spmv(A, x)
        beta = float(np.linalg.norm(r))
        if beta / bn <= rtol:
            return x, KrylovInfo(it, beta / bn, True, applies)
        if it >= maxit:
            return x, KrylovInfo(it, beta / bn, False, applies)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            applies += 1
            w = spmv(A, Z[j])
            it += 1
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            if abs(g[j + 1]) / bn <= rtol or it >= maxit:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + Z[:k].T @ y


def bicgstab(A: CSR, b: np.ndarray, M, rtol: float = 1e-10, maxit: int = 10000, x0=None):
    """Right-preconditioned BiCGSTAB (van der Vorst), shadow residual r0,
    stopping on the true residual ||b - A x|| / ||b|| <= rtol.  One iteration
    applies the preconditioner twice."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return np.zeros(n), KrylovInfo(0, 0.0, True, 0)
    it = 0
    applies = 0
    while True:
        r = b - spmv(A, x)
        if np.linalg.norm(r) / bn <= rtol:
            return x, KrylovInfo(it, float(np.linalg.norm(r) / bn), True, applies)
        if it >= maxit:
            return x, KrylovInfo(it, float(np.linalg.norm(r) / bn), False, applies)
        rh = r.copy()
        rho_old = alpha = omega = 1.0
        v = np.zeros(n)
        p = np.zeros(n)
        restart = False
        while it < maxit:
            rho = float(np.dot(rh, r))
            if rho == 0.0:
                restart = True
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = M(p)
            applies += 1
            v = spmv(A, ph)
            alpha = rho / float(np.dot(rh, v))
            s = r - alpha * v
            it += 1
            if np.linalg.norm(s) / bn <= rtol:
                x = x + alpha * ph
                restart = True
                break
            sh = M(s)
            applies += 1
            t = spmv(A, sh)
            tt = float(np.dot(t, t))
            omega = float(np.dot(t, s)) / tt if tt != 0.0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            if np.linalg.norm(r) / bn <= rtol or omega == 0.0:
                restart = True
                break
            rho_old = rho
        if not restart and it >= maxit:
            continue
