"""Pin of ILUT(p, tau) between its limits (Section 3, ILUT(p, tol)).

tests/golden/ilut_6x6_p2_tau0125.txt holds a 6x6 matrix and its ILUT(2, 1/8)
factors derived by hand, step by step, in the file's comments.  The matrix is
chosen so that each of these rules changes the result: a multiplier dropped
only after its division by the pivot, a fill entry dropped by the final
threshold test, a row whose p largest and p smallest candidates differ, a
magnitude tie at the p-th place (kept: the smaller column) and an entry
exactly at the threshold (kept).  The oracle and the product's host
factorization must both reproduce the factors bit for bit (every value is
dyadic, so the arithmetic is exact), and copies of the oracle with one rule
broken on purpose (compiled here, on the CPU) must fail the pin.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import paper_1606_00541_amd as H
from synth import CSR

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ilut_6x6_p2_tau0125.txt")
ORC_C = os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle", "orc.c")


def _load():
    n = p = None
    tau = None
    ent = {"A": [], "L": [], "U": []}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            f = line.split()
            if f[0] == "n":
                n = int(f[1])
            elif f[0] == "p":
                p = int(f[1])
            elif f[0] == "tau":
                tau = float(f[1])
            else:
                ent[f[0]].append((int(f[1]), int(f[2]), float(f[3])))

    def csr(entries, unit_last=False):
        rows = [[] for _ in range(n)]
        for i, j, v in entries:
            rows[i].append((j, v))
        if unit_last:
            for i in range(n):
                rows[i].append((i, 1.0))
        rp = np.zeros(n + 1, np.int32)
        ci, vv = [], []
        for i in range(n):
            for j, v in rows[i]:
                ci.append(j)
                vv.append(v)
            rp[i + 1] = len(ci)
        return CSR(n, rp, np.array(ci, np.int32), np.array(vv, np.float64))

    return n, p, tau, csr(ent["A"]), csr(ent["L"], unit_last=True), csr(ent["U"])


def _same(X, Y):
    return (np.array_equal(X.rowptr, Y.rowptr) and np.array_equal(X.col, Y.col)
            and np.array_equal(X.val, Y.val))


def test_fixture_is_consistent():
    n, p, tau, A, L, U = _load()
    assert n == 6 and p == 2 and tau == 0.125
    # at most p entries per part, rows sorted, L unit lower, U diagonal first
    for i in range(n):
        lc = L.col[L.rowptr[i]:L.rowptr[i + 1]]
        uc = U.col[U.rowptr[i]:U.rowptr[i + 1]]
        assert len(lc) - 1 <= p and len(uc) - 1 <= p
        assert lc[-1] == i and np.all(lc[:-1] < i) and np.all(np.diff(lc) > 0)
        assert uc[0] == i and np.all(np.diff(uc) > 0)


def test_oracle_ilut_matches_hand_derivation():
    _, p, tau, A, Lg, Ug = _load()
    L, U = oracle.ilut(A, p, tau)
    assert _same(L, Lg), (L.col, L.val)
    assert _same(U, Ug), (U.col, U.val)


def test_host_ilut_matches_hand_derivation():
    _, p, tau, A, Lg, Ug = _load()
    f = H.ilu_setup(A, "ilut", p=p, tol=tau, tune=H.tune_default(host_only=1))
    for which, G in ((0, Lg), (1, Ug)):
        rp, ci, v = H.ilu_factor(f, which)
        assert np.array_equal(rp, G.rowptr) and np.array_equal(ci, G.col) and np.array_equal(v, G.val)


# (name, [(text in orc.c, replacement, expected number of occurrences)])
_CAND_CMP = ("    if (x->mag > y->mag) return -1;\n    if (x->mag < y->mag) return 1;\n"
             "    return (x->col < y->col) ? -1 : (x->col > y->col);")
MUTANTS = {
    "keep_p_smallest": [(_CAND_CMP, "    if (x->mag < y->mag) return -1;\n    if (x->mag > y->mag) return 1;\n"
                         "    return (x->col < y->col) ? -1 : (x->col > y->col);", 1)],
    "ties_to_larger_column": [(_CAND_CMP, _CAND_CMP.replace("(x->col < y->col) ? -1 : (x->col > y->col)",
                                                            "(x->col > y->col) ? -1 : (x->col < y->col)"), 1)],
    "drop_before_division": [("            double wk = w[k] / ukk;\n"
                              "            if (fabs(wk) < tau_i) { w[k] = 0.0; continue; }",
                              "            if (fabs(w[k]) < tau_i) { w[k] = 0.0; continue; }\n"
                              "            double wk = w[k] / ukk;", 1)],
    "threshold_entry_dropped": [("if (fabs(wk) < tau_i)", "if (fabs(wk) <= tau_i)", 1),
                                ("fabs(w[j]) >= tau_i", "fabs(w[j]) > tau_i", 2)],
    "no_final_threshold_test": [("w[j] != 0.0 && fabs(w[j]) >= tau_i", "w[j] != 0.0", 2)],
    "no_division_by_pivot": [("double wk = w[k] / ukk;", "double wk = w[k]; (void)ukk;", 1)],
    "max_norm_threshold": [("nrm = nrm + v[q] * v[q];", "nrm = fmax(nrm, fabs(v[q]));", 1),
                           ("double tau_i = tau * sqrt(nrm);", "double tau_i = tau * nrm;", 1)],
}


def _mutant_lib(name, tmp):
    src = open(ORC_C).read()
    for old, new, count in MUTANTS[name]:
        assert src.count(old) == count, (name, old)
        src = src.replace(old, new)
    c = os.path.join(tmp, name + ".c")
    so = os.path.join(tmp, name + ".so")
    with open(c, "w") as fh:
        fh.write(src)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99", "-o", so, c, "-lm"],
                   check=True)
    lib = ctypes.CDLL(so)
    i32, vp = ctypes.c_int32, ctypes.c_void_p
    lib.orc_ilut.restype = ctypes.c_int
    lib.orc_ilut.argtypes = [i32, vp, vp, vp, i32, ctypes.c_double] + [vp] * 6
    lib.orc_free.argtypes = [vp]
    return lib


def _run_mutant(lib, A, p, tau):
    n = A.n
    rp = np.ascontiguousarray(A.rowptr, np.int32)
    ci = np.ascontiguousarray(A.col, np.int32)
    v = np.ascontiguousarray(A.val, np.float64)
    outs = [ctypes.c_void_p() for _ in range(6)]
    rc = lib.orc_ilut(n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, p, tau, *[ctypes.byref(o) for o in outs])
    if rc != 0:
        return None

    def take(ptr, cnt, dt):
        a = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(np.ctypeslib.as_ctypes_type(dt))), (cnt,)).copy()
        lib.orc_free(ptr)
        return a

    lrp = take(outs[0], n + 1, np.int32)
    lci, lv = take(outs[1], int(lrp[-1]), np.int32), take(outs[2], int(lrp[-1]), np.float64)
    urp = take(outs[3], n + 1, np.int32)
    uci, uv = take(outs[4], int(urp[-1]), np.int32), take(outs[5], int(urp[-1]), np.float64)
    return (lrp, lci, lv), (urp, uci, uv)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_the_pin(name):
    _, p, tau, A, Lg, Ug = _load()
    with tempfile.TemporaryDirectory() as tmp:
        lib = _mutant_lib(name, tmp)
        got = _run_mutant(lib, A, p, tau)
    if got is None:
        return  # the mistake makes the factorization fail outright
    (lrp, lci, lv), (urp, uci, uv) = got
    # golden L without its unit diagonal, in the oracle's C output form
    keep = Lg.col != np.repeat(np.arange(Lg.n), np.diff(Lg.rowptr))
    strict_rp = np.concatenate([[0], np.cumsum(np.diff(Lg.rowptr) - 1)]).astype(np.int32)
    same_l = np.array_equal(lrp, strict_rp) and np.array_equal(lci, Lg.col[keep]) and np.array_equal(lv, Lg.val[keep])
    same_u = np.array_equal(urp, Ug.rowptr) and np.array_equal(uci, Ug.col) and np.array_equal(uv, Ug.val)
    assert not (same_l and same_u), name + " reproduces the golden factors"


def test_unmutated_copy_reproduces_the_pin():
    """The harness above, with no mutation, gives the golden factors (so a
    mutant's failure is the mutation's doing)."""
    _, p, tau, A, Lg, Ug = _load()
    with tempfile.TemporaryDirectory() as tmp:
        so = os.path.join(tmp, "plain.so")
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99", "-o", so, ORC_C, "-lm"],
                       check=True)
        lib = ctypes.CDLL(so)
        i32, vp = ctypes.c_int32, ctypes.c_void_p
        lib.orc_ilut.restype = ctypes.c_int
        lib.orc_ilut.argtypes = [i32, vp, vp, vp, i32, ctypes.c_double] + [vp] * 6
        lib.orc_free.argtypes = [vp]
        (lrp, lci, lv), (urp, uci, uv) = _run_mutant(lib, A, p, tau)
    assert np.array_equal(urp, Ug.rowptr) and np.array_equal(uci, Ug.col) and np.array_equal(uv, Ug.val)
    assert int(lrp[-1]) == Lg.nnz - Lg.n
