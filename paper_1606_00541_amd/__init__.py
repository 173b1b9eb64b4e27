"""Python binding of libhec (include/hec.h): argument marshalling only.

Every computation runs inside libhec: host analysis and factorization in its
C++ part, every solve, preconditioner application and Krylov iteration in its
gfx950 HIP kernels.  Vectors are PyTorch CUDA tensors (device memory and
streams only); matrices are any object with ``n``, ``rowptr``, ``col`` and
``val`` attributes (CSR, 0-based, rows sorted).  The first call loads the
compiled library and raises if it is missing; there is no fallback path.

PyTorch ships its own HIP runtime.  The library is loaded after torch so that
both resolve to that one runtime (two HIP runtimes in one process do not
share devices, streams or allocations).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhec.so")

# hec_status_t
HEC_OK = 0
STATUS_NAMES = {
    0: "OK", 1: "INVALID_ARG", 2: "NOT_TRIANGULAR", 3: "UNSORTED", 4: "MISSING_DIAG", 5: "ZERO_PIVOT",
    6: "ALLOC", 7: "HIP", 8: "NOT_CONVERGED", 9: "BREAKDOWN", 10: "CAPACITY", 11: "TIMEOUT", 12: "NO_DEVICE",
}
HEC_F64, HEC_F32 = 0, 1
HEC_LOWER, HEC_UPPER = 0, 1
SCHED = {"auto": 0, "level_launch": 1, "level_persistent": 2, "owner_persistent": 3}
ILU_KIND = {"ilu0": 0, "iluk": 1, "ilut": 2}
KRYLOV = {"gmres": 0, "fgmres": 1, "bicgstab": 2}
PRECOND = {"none": 0, "ilu": 1, "ras": 2}


class HecError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code
        self.name = STATUS_NAMES.get(code, str(code))


class Tune(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in (
        "ell_width", "schedule", "num_groups", "merge_rows", "group_lanes", "long_row", "part_rows",
        "host_only", "max_nrhs", "block_threads", "chunk_rows", "partition", "kernel_variant")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KrylovInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("precond_applies", ctypes.c_int32), ("relres", ctypes.c_double)]


class TriStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in (
        "n", "nlev", "ell_width", "ld", "num_groups", "nsteps", "nexport", "schedule")] + [
        ("nnz_offdiag", ctypes.c_int64), ("nnz_tail", ctypes.c_int64), ("lds_rows", ctypes.c_int64),
        ("nremote", ctypes.c_int64), ("unit_diag", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("crit_hops", ctypes.c_int32), ("dataflow", ctypes.c_int32), ("syncfree", ctypes.c_int32),
        ("queue", ctypes.c_int32), ("sysq", ctypes.c_int32)]


class Precond(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("handle", ctypes.c_void_p)]


# Every function declared in include/hec.h with its argument types.
_vp, _i32, _i64, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_P = ctypes.POINTER
SIGNATURES = {
    "hec_last_error": (ctypes.c_char_p, []),
    "hec_tune_default": (_i32, [_P(Tune)]),
    "hec_from_csr": (_i32, [_i32, _vp, _vp, _vp, _i32, _i32, _P(_vp)]),
    "hec_spmv": (_i32, [_vp, _vp, _vp, _i32, _vp]),
    "hec_matrix_export": (_i32, [_vp, _P(_i32), _P(_i32), _P(_i64), _vp, _vp, _vp, _vp, _vp]),
    "hec_matrix_destroy": (None, [_vp]),
    "tri_analyze": (_i32, [_i32, _vp, _vp, _vp, _i32, _i32, _i32, _P(Tune), _P(_vp)]),
    "tri_plan_info": (_i32, [_vp, _P(_i32), _P(_i32), _vp, _vp]),
    "tri_plan_hec": (_i32, [_vp, _P(_i32), _P(_i32), _P(_i64), _vp, _vp, _vp, _vp, _vp]),
    "tri_plan_stats": (_i32, [_vp, _P(TriStats)]),
    "tri_plan_layout": (_i32, [_vp, _vp, _vp]),
    "tri_plan_trace": (_i32, [_vp, _vp, _i32]),
    "tri_plan_set_wait_limit": (_i32, [_vp, ctypes.c_uint32]),
    "tri_plan_check": (_i32, [_vp]),
    "tri_solve_lower": (_i32, [_vp, _vp, _vp, _i32, _i32, _vp]),
    "tri_solve_upper": (_i32, [_vp, _vp, _vp, _i32, _i32, _vp]),
    "tri_plan_destroy": (None, [_vp]),
    "ilu_setup": (_i32, [_i32, _vp, _vp, _vp, _i32, _i32, _f64, _i32, _i32, _P(Tune), _P(_vp)]),
    "ilu_factor": (_i32, [_vp, _i32, _P(_i64), _vp, _vp, _vp]),
    "ilu_plans": (_i32, [_vp, _P(_vp), _P(_vp)]),
    "ilu_apply": (_i32, [_vp, _vp, _vp, _i32, _i32, _vp]),
    "ilu_apply_noalloc": (_i32, [_vp, _vp, _vp, _i32, _i32, _vp]),
    "ilu_destroy": (None, [_vp]),
    "ilu_refactor": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "ras_setup": (_i32, [_i32, _vp, _vp, _vp, _i32, _vp, _i32, _i32, _P(Tune), _P(_vp)]),
    "ras_setup_ilu": (_i32, [_i32, _vp, _vp, _vp, _i32, _vp, _i32, _i32, _i32, ctypes.c_double, _i32, _i32,
                             _P(Tune), _P(_vp)]),
    "ras_apply": (_i32, [_vp, _vp, _vp, _i32, _vp]),
    "ras_info": (_i32, [_vp, _P(_i32), _P(_i64), _vp]),
    "ras_plans": (_i32, [_vp, _P(_vp), _P(_vp)]),
    "ras_destroy": (None, [_vp]),
    "ras_refactor": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "sor_setup": (_i32, [_i32, _vp, _vp, _vp, ctypes.c_double, _P(Tune), _P(_vp)]),
    "sor_apply": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _vp]),
    "sor_destroy": (None, [_vp]),
    "batch_setup": (_i32, [_i32, _vp, _vp, _vp, _i32, _vp, _i32, _i32, _f64, _i32, _i32, _P(Tune), _P(_vp)]),
    "krylov_solve": (_i32, [_vp, Precond, _i32, _i32, _vp, _vp, _i32, _f64, _i32, _vp, _vp]),
    "krylov_solve_batch": (_i32, [_vp, Precond, _i32, _i32, _i32, _vp, _vp, _vp, _i32, _f64, _i32, _vp, _vp]),
    "hec_graph_capture": (_i32, [Precond, _vp, _vp, _i32, _i32, _vp, _P(_vp)]),
    "hec_graph_launch": (_i32, [_vp, _vp]),
    "hec_graph_destroy": (None, [_vp]),
    "tri_autotune": (_i32, [_i32, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _vp, ctypes.c_char_p, _f64, _vp,
                            _P(Tune), _P(_f64)]),
}

_lib = None


def lib():
    """The loaded libhec (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhec.so is not built; run __graft_entry__.build() (or "
                              "python paper_1606_00541_amd/_build.py)")
        try:  # bind libhec to the HIP runtime torch has loaded
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != HEC_OK:
        raise HecError(status, lib().hec_last_error().decode(errors="replace"))


def _np(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dt(dtype) -> int:
    s = str(dtype)
    if s in ("f64", "float64", "torch.float64", "double"):
        return HEC_F64
    if s in ("f32", "float32", "torch.float32", "float"):
        return HEC_F32
    raise ValueError("unsupported dtype %r" % (dtype,))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _vec(t, n):
    """(pointer, nrhs, dtype code) of a CUDA tensor shaped [n] or [n][nrhs]."""
    if not t.is_cuda:
        raise ValueError("vectors must be CUDA tensors")
    if not t.is_contiguous():
        raise ValueError("vectors must be contiguous ([n][nrhs], RHS index fastest)")
    if t.shape[0] != n:
        raise ValueError("vector has %d rows, expected %d" % (t.shape[0], n))
    nrhs = 1 if t.dim() == 1 else int(t.shape[1])
    return ctypes.c_void_p(t.data_ptr()), nrhs, _dt(t.dtype)


def tune_default(**kw) -> Tune:
    t = Tune()
    _check(lib().hec_tune_default(ctypes.byref(t)))
    for k, v in kw.items():
        if k == "schedule" and isinstance(v, str):
            v = SCHED[v]
        setattr(t, k, int(v))
    return t


class _Handle:
    _destroy = None

    def __init__(self, ptr, keep=None):
        self.ptr = ptr
        self._keep = keep

    def __del__(self):
        if self.ptr and self._destroy and _lib is not None:
            getattr(_lib, self._destroy)(self.ptr)
            self.ptr = None


class HecMatrix(_Handle):
    _destroy = "hec_matrix_destroy"


class TriPlan(_Handle):
    _destroy = "tri_plan_destroy"


class _BorrowedPlan(_Handle):
    _destroy = None


class Ilu(_Handle):
    _destroy = "ilu_destroy"


class Ras(_Handle):
    _destroy = "ras_destroy"


class Sor(_Handle):
    _destroy = "sor_destroy"


class Graph(_Handle):
    _destroy = "hec_graph_destroy"


def _csr(A, dtype=np.float64):
    return (int(A.n), _np(A.rowptr, np.int32), _np(A.col, np.int32), _np(A.val, dtype))


# ---- HEC matrix -----------------------------------------------------------

def hec_from_csr(A, dtype="f64", ell_width: int = -1) -> HecMatrix:
    n, rp, ci, v = _csr(A, np.float64 if _dt(dtype) == HEC_F64 else np.float32)
    out = ctypes.c_void_p()
    _check(lib().hec_from_csr(n, _ptr(rp), _ptr(ci), _ptr(v), _dt(dtype), int(ell_width), ctypes.byref(out)))
    m = HecMatrix(out.value)
    m.n = n
    return m


def hec_spmv(A: HecMatrix, x, y, stream=None):
    px, R, dx = _vec(x, A.n)
    py, R2, dy = _vec(y, A.n)
    if R != R2 or dx != HEC_F64 or dy != HEC_F64:
        raise ValueError("hec_spmv takes FP64 vectors of equal shape")
    _check(lib().hec_spmv(A.ptr, px, py, R, _stream(stream)))


def _export(fn, handle, n):
    w, ld, tail = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(fn(handle, ctypes.byref(w), ctypes.byref(ld), ctypes.byref(tail), None, None, None, None, None))
    ec = np.empty(w.value * ld.value, np.int32)
    ev = np.empty(w.value * ld.value, np.float64)
    cp = np.empty(n + 1, np.int32)
    cc = np.empty(tail.value, np.int32)
    cv = np.empty(tail.value, np.float64)
    _check(fn(handle, ctypes.byref(w), ctypes.byref(ld), ctypes.byref(tail), _ptr(ec), _ptr(ev), _ptr(cp),
              _ptr(cc), _ptr(cv)))
    return dict(width=w.value, ld=ld.value, ell_col=ec, ell_val=ev, csr_ptr=cp, csr_col=cc, csr_val=cv)


def hec_matrix_export(A: HecMatrix) -> dict:
    return _export(lib().hec_matrix_export, A.ptr, A.n)


# ---- triangular plans -----------------------------------------------------

def tri_analyze(T, uplo="lower", unit_diag=False, dtype="f64", tune: Tune | None = None) -> TriPlan:
    n, rp, ci, v = _csr(T, np.float64 if _dt(dtype) == HEC_F64 else np.float32)
    out = ctypes.c_void_p()
    up = HEC_UPPER if uplo in ("upper", HEC_UPPER) else HEC_LOWER
    _check(lib().tri_analyze(n, _ptr(rp), _ptr(ci), _ptr(v), _dt(dtype), up, int(bool(unit_diag)),
                             ctypes.byref(tune) if tune is not None else None, ctypes.byref(out)))
    p = TriPlan(out.value)
    p.n = n
    return p


def _plan_n(plan):
    n = ctypes.c_int32()
    _check(lib().tri_plan_info(plan.ptr, ctypes.byref(n), None, None, None))
    return n.value


def tri_plan_info(plan):
    """(nlev, levelptr[nlev+1], perm[n]) of eq. (2)-(3)."""
    n, nlev = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().tri_plan_info(plan.ptr, ctypes.byref(n), ctypes.byref(nlev), None, None))
    lp = np.empty(nlev.value + 1, np.int32)
    perm = np.empty(n.value, np.int32)
    _check(lib().tri_plan_info(plan.ptr, None, None, _ptr(lp), _ptr(perm)))
    return nlev.value, lp, perm


def tri_plan_hec(plan) -> dict:
    return _export(lib().tri_plan_hec, plan.ptr, _plan_n(plan))


def tri_plan_stats(plan) -> dict:
    s = TriStats()
    _check(lib().tri_plan_stats(plan.ptr, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in s._fields_}


def tri_plan_layout(plan):
    n = _plan_n(plan)
    xp = np.empty(n, np.int32)
    ow = np.empty(n, np.int32)
    _check(lib().tri_plan_layout(plan.ptr, _ptr(xp), _ptr(ow)))
    return xp, ow


def tri_plan_trace(plan, trace=None, stride=0):
    """Attach (or with None detach) a device uint64 tensor of
    2*groups*stride entries receiving per-step start/end shader clocks."""
    ptr = ctypes.c_void_p(trace.data_ptr()) if trace is not None else None
    _check(lib().tri_plan_trace(plan.ptr, ptr, int(stride)))


def tri_plan_set_wait_limit(plan, polls=0):
    """Polls before a bounded device-side wait gives up (0 = default)."""
    _check(lib().tri_plan_set_wait_limit(plan.ptr, int(polls)))


def tri_plan_check(plan):
    """Raise HecError(TIMEOUT) if an earlier launch of the plan aborted a wait
    (and clear the flag); the caller synchronizes the stream first."""
    _check(lib().tri_plan_check(plan.ptr))


def tri_solve_lower(plan, b, x, stream=None):
    n = plan.n
    pb, R, db = _vec(b, n)
    px, R2, dx = _vec(x, n)
    if R != R2 or db != dx:
        raise ValueError("b and x must have the same shape and dtype")
    _check(lib().tri_solve_lower(plan.ptr, pb, px, R, db, _stream(stream)))


def tri_solve_upper(plan, b, x, stream=None):
    n = plan.n
    pb, R, db = _vec(b, n)
    px, R2, dx = _vec(x, n)
    if R != R2 or db != dx:
        raise ValueError("b and x must have the same shape and dtype")
    _check(lib().tri_solve_upper(plan.ptr, pb, px, R, db, _stream(stream)))


def tri_autotune(T, uplo="lower", unit_diag=False, dtype="f64", nrhs=1, sys_ptr=None, cache=None,
                 max_seconds=0.0, stream=None):
    """Fastest tuning for solving with T (and its time per solve in us);
    sys_ptr marks independent systems, cache is a JSON-lines file path."""
    n, rp, ci, v = _csr(T, np.float64 if _dt(dtype) == HEC_F64 else np.float32)
    best = Tune()
    us = ctypes.c_double()
    up = HEC_UPPER if uplo in ("upper", HEC_UPPER) else HEC_LOWER
    sp = None if sys_ptr is None else _np(sys_ptr, np.int32)
    nsys = 0 if sp is None else len(sp) - 1
    _check(lib().tri_autotune(n, _ptr(rp), _ptr(ci), _ptr(v), _dt(dtype), up, int(bool(unit_diag)), int(nrhs),
                              nsys, None if sp is None else sp.ctypes.data,
                              None if cache is None else os.fsencode(cache), float(max_seconds),
                              _stream(stream), ctypes.byref(best), ctypes.byref(us)))
    return best, us.value


# ---- ILU / batch / RAS ----------------------------------------------------

def ilu_setup(A, kind="ilu0", k=0, tol=0.0, p=0, factor_dtype="f64", tune: Tune | None = None) -> Ilu:
    n, rp, ci, v = _csr(A)
    out = ctypes.c_void_p()
    _check(lib().ilu_setup(n, _ptr(rp), _ptr(ci), _ptr(v), ILU_KIND[kind], int(k), float(tol), int(p),
                           _dt(factor_dtype), ctypes.byref(tune) if tune is not None else None, ctypes.byref(out)))
    f = Ilu(out.value)
    f.n = n
    return f


def batch_setup(A, sys_ptr, kind="ilu0", k=0, tol=0.0, p=0, factor_dtype="f64", tune: Tune | None = None) -> Ilu:
    n, rp, ci, v = _csr(A)
    sp = _np(sys_ptr, np.int32)
    out = ctypes.c_void_p()
    _check(lib().batch_setup(n, _ptr(rp), _ptr(ci), _ptr(v), int(sp.shape[0] - 1), _ptr(sp), ILU_KIND[kind],
                             int(k), float(tol), int(p), _dt(factor_dtype),
                             ctypes.byref(tune) if tune is not None else None, ctypes.byref(out)))
    f = Ilu(out.value)
    f.n = n
    return f


def ilu_factor(f: Ilu, which: int):
    """Host copy of factor `which` (0 = L with stored unit diagonal, 1 = U)."""
    nnz = ctypes.c_int64()
    _check(lib().ilu_factor(f.ptr, int(which), ctypes.byref(nnz), None, None, None))
    rp = np.empty(f.n + 1, np.int32)
    ci = np.empty(nnz.value, np.int32)
    v = np.empty(nnz.value, np.float64)
    _check(lib().ilu_factor(f.ptr, int(which), ctypes.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v)))
    return rp, ci, v


def ilu_plans(f: Ilu):
    L, U = ctypes.c_void_p(), ctypes.c_void_p()
    _check(lib().ilu_plans(f.ptr, ctypes.byref(L), ctypes.byref(U)))
    pl, pu = _BorrowedPlan(L.value, keep=f), _BorrowedPlan(U.value, keep=f)
    pl.n = pu.n = f.n
    return pl, pu


def ilu_refactor(f: Ilu, A=None, val=None, stream=None):
    """Refactor on the device with new values of A (pattern inside the
    setup's factor pattern).  ``val``: device FP64 tensor of A's values in CSR
    order (default: A's host values, copied to the device).  With A None the
    previous call's pattern is reused and ``val`` is required."""
    import torch

    if A is None:
        if val is None:
            raise ValueError("val is required when A is None")
        rp = ci = None
    else:
        n, rp, ci, v = _csr(A)
        if val is None:
            val = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
        if val.numel() != ci.shape[0]:
            raise ValueError("val must hold nnz(A) values")
    if val.dtype != torch.float64 or not val.is_cuda:
        raise ValueError("val must be a device FP64 tensor")
    val = val.contiguous()
    _check(lib().ilu_refactor(f.ptr, _ptr(rp) if rp is not None else None, _ptr(ci) if ci is not None else None,
                              ctypes.c_void_p(val.data_ptr()), _stream(stream)))


def ilu_apply(f: Ilu, r, z, stream=None):
    pr, R, dr = _vec(r, f.n)
    pz, R2, dz = _vec(z, f.n)
    if R != R2 or dr != dz:
        raise ValueError("r and z must have the same shape and dtype")
    _check(lib().ilu_apply(f.ptr, pr, pz, R, dr, _stream(stream)))


def ilu_apply_noalloc(f: Ilu, r, z, stream=None):
    """ilu_apply through the entry point that allocates nothing (the
    library's fixed device scratch array; nrhs at most the handle's max_nrhs)."""
    pr, R, dr = _vec(r, f.n)
    pz, R2, dz = _vec(z, f.n)
    if R != R2 or dr != dz:
        raise ValueError("r and z must have the same shape and dtype")
    _check(lib().ilu_apply_noalloc(f.ptr, pr, pz, R, dr, _stream(stream)))


def ras_setup(A, nsub, owner, overlap=1, factor_dtype="f64", tune: Tune | None = None) -> Ras:
    n, rp, ci, v = _csr(A)
    ow = _np(owner, np.int32)
    out = ctypes.c_void_p()
    _check(lib().ras_setup(n, _ptr(rp), _ptr(ci), _ptr(v), int(nsub), _ptr(ow), int(overlap), _dt(factor_dtype),
                           ctypes.byref(tune) if tune is not None else None, ctypes.byref(out)))
    s = Ras(out.value)
    s.n = n
    s.nsub = int(nsub)
    return s


def ras_setup_ilu(A, nsub, owner, overlap=0, kind="ilut", k=0, tol=0.0, p=0, factor_dtype="f64",
                  tune: Tune | None = None) -> Ras:
    """Block ILU(k) / block ILUT (overlap 0) or RAS with that subdomain
    factorization (overlap > 0)."""
    n, rp, ci, v = _csr(A)
    ow = _np(owner, np.int32)
    out = ctypes.c_void_p()
    _check(lib().ras_setup_ilu(n, _ptr(rp), _ptr(ci), _ptr(v), int(nsub), _ptr(ow), int(overlap), ILU_KIND[kind],
                               int(k), float(tol), int(p), _dt(factor_dtype),
                               ctypes.byref(tune) if tune is not None else None, ctypes.byref(out)))
    s = Ras(out.value)
    s.n = n
    s.nsub = int(nsub)
    return s


def sor_setup(A, omega=1.0, tune: Tune | None = None) -> Sor:
    """SOR / Gauss-Seidel smoother of A (FP64 plans of D/omega + L and
    D/omega + U, and the two SpMV operators)."""
    n, rp, ci, v = _csr(A)
    out = ctypes.c_void_p()
    _check(lib().sor_setup(n, _ptr(rp), _ptr(ci), _ptr(v), float(omega),
                           ctypes.byref(tune) if tune is not None else None, ctypes.byref(out)))
    s = Sor(out.value)
    s.n = n
    return s


def sor_apply(s: Sor, b, x, sweeps=1, symmetric=False, stream=None):
    """`sweeps` SOR sweeps on x in place (forward, or SSOR when symmetric)."""
    pb, R, db = _vec(b, s.n)
    px, R2, dx = _vec(x, s.n)
    if R != R2 or db != HEC_F64 or dx != HEC_F64:
        raise ValueError("sor_apply takes FP64 b and x of equal shape")
    _check(lib().sor_apply(s.ptr, pb, px, R, int(sweeps), int(bool(symmetric)), _stream(stream)))


def ras_refactor(s: Ras, A=None, val=None, stream=None):
    """Refactor a RAS / block ILU handle on the device with new values of A
    (same pattern); arguments as ilu_refactor."""
    import torch

    if A is None:
        if val is None:
            raise ValueError("val is required when A is None")
        rp = ci = None
    else:
        n, rp, ci, v = _csr(A)
        if val is None:
            val = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
        if val.numel() != ci.shape[0]:
            raise ValueError("val must hold nnz(A) values")
    if val.dtype != torch.float64 or not val.is_cuda:
        raise ValueError("val must be a device FP64 tensor")
    val = val.contiguous()
    _check(lib().ras_refactor(s.ptr, _ptr(rp) if rp is not None else None, _ptr(ci) if ci is not None else None,
                              ctypes.c_void_p(val.data_ptr()), _stream(stream)))


def ras_apply(s: Ras, r, z, stream=None):
    pr, R, dr = _vec(r, s.n)
    pz, R2, dz = _vec(z, s.n)
    if R != R2 or dr != HEC_F64 or dz != HEC_F64:
        raise ValueError("ras_apply takes FP64 vectors of equal shape")
    _check(lib().ras_apply(s.ptr, pr, pz, R, _stream(stream)))


def ras_info(s: Ras):
    nsub, tot = ctypes.c_int32(), ctypes.c_int64()
    sizes = np.empty(s.nsub, np.int32)
    _check(lib().ras_info(s.ptr, ctypes.byref(nsub), ctypes.byref(tot), _ptr(sizes)))
    return nsub.value, tot.value, sizes


def ras_plans(s: Ras):
    L, U = ctypes.c_void_p(), ctypes.c_void_p()
    _check(lib().ras_plans(s.ptr, ctypes.byref(L), ctypes.byref(U)))
    n = int(ras_info(s)[1])
    pl, pu = _BorrowedPlan(L.value, keep=s), _BorrowedPlan(U.value, keep=s)
    pl.n = pu.n = n
    return pl, pu


def _precond(M) -> Precond:
    if M is None:
        return Precond(PRECOND["none"], None)
    if isinstance(M, Ilu):
        return Precond(PRECOND["ilu"], M.ptr)
    if isinstance(M, Ras):
        return Precond(PRECOND["ras"], M.ptr)
    raise TypeError("preconditioner must be None, Ilu or Ras")


# ---- Krylov ---------------------------------------------------------------

def krylov_solve(A: HecMatrix, M, b, x, method="fgmres", m=30, rtol=1e-10, maxit=10000, stream=None,
                 raise_on_fail=False):
    """Solve A x = b (x holds x0).  Returns (status, [KrylovInfo per RHS])."""
    pb, R, db = _vec(b, A.n)
    px, R2, dx = _vec(x, A.n)
    if R != R2 or db != HEC_F64 or dx != HEC_F64:
        raise ValueError("krylov_solve takes FP64 b and x of equal shape")
    infos = (KrylovInfo * R)()
    st = lib().krylov_solve(A.ptr, _precond(M), KRYLOV[method], int(m), pb, px, R, float(rtol), int(maxit),
                            ctypes.cast(infos, ctypes.c_void_p), _stream(stream))
    if st != HEC_OK and (raise_on_fail or st not in (8, 9)):
        _check(st)
    return st, list(infos)


def krylov_solve_batch(A: HecMatrix, M, sys_ptr, b, x, method="fgmres", m=30, rtol=1e-10, maxit=10000,
                       stream=None, raise_on_fail=False):
    """Solve the independent systems of a block-diagonal A (blocks given by
    sys_ptr) together, each (system, rhs) pair as its own Krylov problem.
    Returns (status, [KrylovInfo per pair, system-major])."""
    pb, R, db = _vec(b, A.n)
    px, R2, dx = _vec(x, A.n)
    if R != R2 or db != HEC_F64 or dx != HEC_F64:
        raise ValueError("krylov_solve_batch takes FP64 b and x of equal shape")
    sp = _np(sys_ptr, np.int32)
    nsys = len(sp) - 1
    infos = (KrylovInfo * (nsys * R))()
    st = lib().krylov_solve_batch(A.ptr, _precond(M), KRYLOV[method], int(m), nsys, sp.ctypes.data, pb, px, R,
                                  float(rtol), int(maxit), ctypes.cast(infos, ctypes.c_void_p), _stream(stream))
    if st != HEC_OK and (raise_on_fail or st not in (8, 9)):
        _check(st)
    return st, list(infos)


# ---- graphs ---------------------------------------------------------------

def hec_graph_capture(M, r, z, stream=None) -> Graph:
    n = M.n
    pr, R, dr = _vec(r, n)
    pz, R2, dz = _vec(z, n)
    if R != R2 or dr != dz:
        raise ValueError("r and z must have the same shape and dtype")
    out = ctypes.c_void_p()
    _check(lib().hec_graph_capture(_precond(M), pr, pz, R, dr, _stream(stream), ctypes.byref(out)))
    return Graph(out.value, keep=(M, r, z))


def hec_graph_launch(g: Graph, stream=None):
    _check(lib().hec_graph_launch(g.ptr, _stream(stream)))
