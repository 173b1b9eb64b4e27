"""CPU tests of the C ABI: the library loads and exports every function the
header declares, and the host-side analysis (Algorithm 1), factorizations
and RAS setup agree bit for bit with the oracle.  No GPU is touched: plans
are built with the host-only tuning flag."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from synth import CSR

import paper_1606_00541_amd as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = H.tune_default(host_only=1)


def _header_functions():
    text = open(os.path.join(ROOT, "include", "hec.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    names = _header_functions()
    assert len(names) >= 30
    lib = H.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(H.SIGNATURES), set(names) ^ set(H.SIGNATURES)


def test_tune_defaults_and_validation():
    t = H.tune_default()
    assert t.ell_width == -1 and t.schedule == 0 and t.block_threads == 256 and t.max_nrhs == 1
    L = synth.random_lower(50, 0.05, seed=1)
    with pytest.raises(H.HecError) as e:
        H.tri_analyze(L, tune=H.tune_default(host_only=1, block_threads=100))
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(H.HecError):
        H.tri_analyze(L, tune=H.tune_default(host_only=1, group_lanes=3))
    with pytest.raises(H.HecError):
        H.tri_analyze(L, tune=H.tune_default(host_only=1, kernel_variant=7))
    with pytest.raises(H.HecError):  # the queue-mode dataflow kernel runs the owner schedule only
        H.tri_analyze(L, tune=H.tune_default(host_only=1, kernel_variant=6, schedule="level_launch"))
    with pytest.raises(H.HecError):  # the barrier-free kernel runs the level-ordered layout only
        H.tri_analyze(L, tune=H.tune_default(host_only=1, kernel_variant=5, schedule="owner_persistent"))
    p = H.tri_analyze(L, tune=H.tune_default(host_only=1, kernel_variant=5))
    assert H.tri_plan_stats(p)["schedule"] == 1
    with pytest.raises(H.HecError):
        H.tri_analyze(L, tune=H.tune_default(host_only=1, block_threads=256, chunk_rows=768))
    # an owner plan with the default chunk size builds (steps are cut to chunks)
    p = H.tri_analyze(L, tune=H.tune_default(host_only=1, schedule="owner_persistent", chunk_rows=0))
    assert H.tri_plan_stats(p)["nsteps"] > 0


def _transpose(T):
    m = T.to_scipy().T.tocsr()
    m.sort_indices()
    return CSR(T.n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())


def _cases():
    A2 = synth.poisson2d(64)
    L2, U2 = oracle.ilu0(A2)
    A3 = synth.diffusion3d(12, 11, 10, 2.0, seed=3)
    Lt, Ut = oracle.ilut(A3, 10, 1e-3)
    Lr = synth.random_lower(700, 0.01, seed=7, dense_row=350)
    return [("poisson64 L", L2, False, True), ("poisson64 U", U2, True, False),
            ("ilut L", Lt, False, True), ("ilut U", Ut, True, False),
            ("random L", Lr, False, False), ("random U", _transpose(Lr), True, False)]


@pytest.mark.parametrize("case", range(6))
@pytest.mark.parametrize("sched", ["level_launch", "level_persistent", "owner_persistent", "owner_dataflow"])
def test_levels_map_and_hec_bit_exact(case, sched):
    name, T, upper, unit = _cases()[case]
    if sched == "owner_dataflow":
        t = H.tune_default(host_only=1, schedule="owner_persistent", kernel_variant=4, num_groups=16)
    elif sched == "owner_persistent":  # the LDS-chunked owner kernel's layout
        t = H.tune_default(host_only=1, schedule=sched, kernel_variant=2, num_groups=16)
    else:
        t = H.tune_default(host_only=1, schedule=sched, num_groups=16)
    p = H.tri_analyze(T, "upper" if upper else "lower", unit_diag=unit, tune=t)
    nlev, lp, perm = H.tri_plan_info(p)
    lev, nl = oracle.levels(T, upper=upper)
    lp2, perm2, iperm2 = oracle.level_schedule(lev, nl, upper=upper)
    assert nlev == nl
    assert np.array_equal(lp, lp2) and np.array_equal(perm, perm2)
    # HEC round trip: rebuilding CSR from the exported HEC gives L' exactly
    h = H.tri_plan_hec(p)
    R = oracle.hec_to_csr(T.n, h["width"], h["ld"], h["ell_col"], h["ell_val"], h["csr_ptr"], h["csr_col"],
                          h["csr_val"])
    Tp = oracle.reorder(T, perm2, iperm2)
    if unit:  # the unit diagonal is stored as 1.0 in the CSR part
        assert np.all(R.val[R.rowptr[1:] - 1] == 1.0)
        assert np.array_equal(R.col, Tp.col) and np.array_equal(R.rowptr, Tp.rowptr)
        off = np.ones(R.nnz, bool)
        off[R.rowptr[1:] - 1] = False
        assert np.array_equal(R.val[off], Tp.val[off])
    else:
        assert np.array_equal(R.rowptr, Tp.rowptr) and np.array_equal(R.col, Tp.col)
        assert np.array_equal(R.val, Tp.val)
    # every CSR row holds at least the diagonal; ELL is column-major, aligned
    assert np.all(np.diff(h["csr_ptr"]) >= 1) and h["ld"] % 64 == 0 and h["ld"] >= T.n
    # the device layout is a permutation processed in dependency order
    xperm, owner = H.tri_plan_layout(p)
    assert np.array_equal(np.sort(xperm), np.arange(T.n))
    if sched == "owner_persistent":
        for g in np.unique(owner):
            rows = xperm[owner == g]
            assert np.all(np.diff(lev[rows]) >= 0)  # level order inside a group
    if sched.startswith("owner"):
        # every dependency inside a group comes earlier in the group's order
        pos = np.empty(T.n, np.int64)
        pos[xperm] = np.arange(T.n)
        rows = np.repeat(np.arange(T.n), np.diff(T.rowptr))
        dep = T.col != rows
        i, j = rows[dep], T.col[dep]
        same = owner[pos[i]] == owner[pos[j]]
        assert np.all(pos[j][same] < pos[i][same])
    st = H.tri_plan_stats(p)
    assert st["nlev"] == nl and st["n"] == T.n


def test_auto_ell_width_is_median():
    A = synth.poisson3d(10)
    L, U = oracle.ilu0(A)
    p = H.tri_analyze(L, unit_diag=True, tune=HOST)
    assert H.tri_plan_stats(p)["ell_width"] == 3
    assert H.tri_plan_stats(p)["nnz_tail"] == 0


@pytest.mark.parametrize("bad,code", [
    ("unsorted", "UNSORTED"), ("upper_entry", "NOT_TRIANGULAR"), ("no_diag", "MISSING_DIAG"),
    ("zero_diag", "ZERO_PIVOT"), ("nan_diag", "ZERO_PIVOT"), ("col_range", "INVALID_ARG")])
def test_invalid_inputs_are_reported(bad, code):
    n = 4
    rp = np.array([0, 1, 3, 5, 7], np.int32)
    ci = np.array([0, 0, 1, 1, 2, 2, 3], np.int32)
    v = np.array([2.0, 1.0, 2.0, 1.0, 2.0, 1.0, 2.0])
    if bad == "unsorted":
        ci = np.array([0, 1, 0, 1, 2, 2, 3], np.int32)
    elif bad == "upper_entry":
        ci = np.array([0, 0, 2, 1, 2, 2, 3], np.int32)
    elif bad == "no_diag":
        ci = np.array([0, 0, 1, 0, 1, 2, 3], np.int32)
    elif bad == "zero_diag":
        v[2] = 0.0
    elif bad == "nan_diag":
        v[2] = np.nan
    elif bad == "col_range":
        ci[3] = 9
    with pytest.raises(H.HecError) as e:
        H.tri_analyze(CSR(n, rp, ci, v), "lower", tune=HOST)
    assert e.value.name == code


@pytest.mark.parametrize("kind,args", [("ilu0", {}), ("iluk", {"k": 1}), ("iluk", {"k": 3}),
                                       ("ilut", {"p": 10, "tol": 1e-3}), ("ilut", {"p": 2, "tol": 1e-2})])
def test_factorizations_bit_exact(kind, args):
    A = synth.diffusion3d(9, 8, 7, 2.0, seed=11)
    f = H.ilu_setup(A, kind, tune=HOST, **args)
    if kind == "ilu0":
        L, U = oracle.ilu0(A)
    elif kind == "iluk":
        L, U = oracle.iluk(A, args["k"])
    else:
        L, U = oracle.ilut(A, args["p"], args["tol"])
    for which, T in ((0, L), (1, U)):
        rp, ci, v = H.ilu_factor(f, which)
        assert np.array_equal(rp, T.rowptr) and np.array_equal(ci, T.col) and np.array_equal(v, T.val)


def test_factorization_errors():
    A = synth.poisson2d(4)
    v = A.val.copy()
    v[0] = 0.0  # zero first pivot
    with pytest.raises(H.HecError) as e:
        H.ilu_setup(CSR(A.n, A.rowptr, A.col, v), "ilu0", tune=HOST)
    assert e.value.name == "ZERO_PIVOT"


def test_ras_layout_matches_oracle():
    A = synth.poisson3d(10)
    owner, _ = synth.subdomain_cuts(A.n, 5, 100, 300, seed=4)
    s = H.ras_setup(A, 5, owner, overlap=1, tune=HOST)
    doms = oracle.ras_setup(A, owner, 5, overlap=1)
    nsub, tot, sizes = H.ras_info(s)
    assert nsub == 5 and tot == sum(len(d.ext) for d in doms)
    assert list(sizes) == [len(d.ext) for d in doms]



def test_block_ilu_layout_and_errors():
    A = synth.diffusion3d(8, 8, 6, 1.0, seed=3)
    owner = synth.grid_bisection(8, 8, 6, 6)
    s = H.ras_setup_ilu(A, 6, owner, overlap=0, kind="ilut", p=7, tol=0.1, tune=HOST)
    nsub, tot, sizes = H.ras_info(s)
    assert nsub == 6 and tot == A.n and list(sizes) == list(np.bincount(owner))
    s1 = H.ras_setup_ilu(A, 6, owner, overlap=1, kind="iluk", k=1, tune=HOST)
    doms = oracle.ras_setup(A, owner, 6, overlap=1, kind="iluk", k=1)
    assert list(H.ras_info(s1)[2]) == [len(d.ext) for d in doms]
    for kw in ({"kind": "iluk", "k": -1}, {"kind": "ilut", "p": -1}, {"kind": "ilut", "tol": -1.0}):
        with pytest.raises(H.HecError) as e:
            H.ras_setup_ilu(A, 6, owner, tune=HOST, **kw)
        assert e.value.name == "INVALID_ARG"
    n, rp, ci, v = H._csr(A)
    out = ctypes.c_void_p()
    rc = H.lib().ras_setup_ilu(n, H._ptr(rp), H._ptr(ci), H._ptr(v), 6, H._ptr(owner.astype(np.int32)), 0, 7, 0,
                               0.0, 0, 0, ctypes.byref(HOST), ctypes.byref(out))
    assert H.STATUS_NAMES[rc] == "INVALID_ARG"




def test_refactor_needs_a_device_and_a_fixed_pattern_kind():
    A = synth.poisson2d(6)
    n, rp, ci, v = H._csr(A)
    for kind, code in (("ilu0", "NO_DEVICE"), ("ilut", "INVALID_ARG")):
        f = H.ilu_setup(A, kind, p=4, tol=1e-2, tune=HOST)
        rc = H.lib().ilu_refactor(f.ptr, H._ptr(rp), H._ptr(ci), None, None)
        assert H.STATUS_NAMES[rc] == code
    owner = synth.grid_bisection(6, 6, 1, 4)
    for kind, code in (("iluk", "NO_DEVICE"), ("ilut", "INVALID_ARG")):
        s = H.ras_setup_ilu(A, 4, owner, overlap=1, kind=kind, k=1, p=4, tol=1e-2, tune=HOST)
        rc = H.lib().ras_refactor(s.ptr, H._ptr(rp), H._ptr(ci), None, None)
        assert H.STATUS_NAMES[rc] == code


def test_sor_setup_validation():
    A = synth.diffusion2d(6, 5, 1.0, seed=2)
    s = H.sor_setup(A, 1.2, tune=HOST)
    with pytest.raises(H.HecError) as e:  # host-only setup has no device plans
        H._check(H.lib().sor_apply(s.ptr, None, None, 1, 1, 0, None))
    assert e.value.name == "NO_DEVICE"
    for om in (0.0, 2.0, -1.0):
        with pytest.raises(H.HecError) as e:
            H.sor_setup(A, om, tune=HOST)
        assert e.value.name == "INVALID_ARG"
    v = A.val.copy()
    diag = A.col == np.repeat(np.arange(A.n), np.diff(A.rowptr))
    v[np.flatnonzero(diag)[3]] = 0.0
    with pytest.raises(H.HecError) as e:
        H.sor_setup(CSR(A.n, A.rowptr, A.col, v), 1.0, tune=HOST)
    assert e.value.name == "ZERO_PIVOT"
    keep = ~(diag & (np.repeat(np.arange(A.n), np.diff(A.rowptr)) == 4))
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))[keep]
    rp = np.zeros(A.n + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=A.n), out=rp[1:])
    with pytest.raises(H.HecError) as e:
        H.sor_setup(CSR(A.n, rp, A.col[keep], A.val[keep]), 1.0, tune=HOST)
    assert e.value.name == "MISSING_DIAG"


def test_auto_tuning_picks_the_dataflow_kernel_when_it_fits():
    A = synth.poisson3d(12)
    L, _ = oracle.ilu0(A)
    st = H.tri_plan_stats(H.tri_analyze(L, unit_diag=True, tune=HOST))
    assert st["schedule"] == 3 and st["dataflow"] == 1
    # one group cannot hold every row in LDS: the level-ordered layout, run by
    # the barrier-free kernel when levels are narrow ...
    A = synth.poisson2d(160)
    L, _ = oracle.ilu0(A)
    st = H.tri_plan_stats(H.tri_analyze(L, unit_diag=True, tune=H.tune_default(host_only=1, num_groups=1)))
    assert st["schedule"] == 1 and st["dataflow"] == 0 and st["syncfree"] == 1
    # ... and by one launch per level when they are wide (2^20 items and more)
    n = (1 << 20) + 64
    D = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 2.0))
    st = H.tri_plan_stats(H.tri_analyze(D, tune=H.tune_default(host_only=1, num_groups=1)))
    assert st["schedule"] == 1 and st["nlev"] == 1 and st["syncfree"] == 0
    # the part queue runs on request (kernel_variant 6)
    st = H.tri_plan_stats(H.tri_analyze(L, unit_diag=True, tune=H.tune_default(
        host_only=1, schedule="owner_persistent", kernel_variant=6)))
    assert st["schedule"] == 3 and st["dataflow"] == 1 and st["queue"] == 1 and st["num_groups"] > 1
    # an explicit owner schedule falls back to the LDS-chunked owner kernel
    st = H.tri_plan_stats(H.tri_analyze(L, unit_diag=True, tune=H.tune_default(
        host_only=1, schedule="owner_persistent", num_groups=1)))
    assert st["schedule"] == 3 and st["dataflow"] == 0


def test_dataflow_plan_limits():
    L = synth.random_lower(400, 0.01, seed=2)
    # the dataflow kernel sizes its steps for max_nrhs; more than 64 cannot fit a wavefront
    with pytest.raises(H.HecError):
        H.tri_analyze(L, tune=H.tune_default(host_only=1, schedule="owner_persistent", kernel_variant=4,
                                             max_nrhs=65))
    with pytest.raises(H.HecError):
        H.tri_analyze(L, tune=H.tune_default(host_only=1, schedule="owner_persistent", kernel_variant=4,
                                             block_threads=704))
    # one group holding every row of a large system does not fit in LDS
    A = synth.poisson2d(160)
    Lp, _ = oracle.ilu0(A)
    with pytest.raises(H.HecError) as e:
        H.tri_analyze(Lp, unit_diag=True, tune=H.tune_default(host_only=1, schedule="owner_persistent",
                                                              kernel_variant=4, num_groups=1))
    assert e.value.name == "CAPACITY"
    p = H.tri_analyze(Lp, unit_diag=True, tune=H.tune_default(host_only=1, schedule="owner_persistent",
                                                              kernel_variant=4, num_groups=8))
    st = H.tri_plan_stats(p)
    assert st["num_groups"] == 8 and st["nsteps"] >= st["nlev"]


def test_owner_partitions():
    A = synth.poisson3d(24)
    L, _ = oracle.ilu0(A)
    stats = {}
    for part in (1, 2, 3):
        t = H.tune_default(host_only=1, schedule="owner_persistent", partition=part, num_groups=64)
        stats[part] = H.tri_plan_stats(H.tri_analyze(L, unit_diag=True, tune=t))
    # grid blocks: far fewer group-to-group handoffs and exported rows than slabs
    assert stats[3]["crit_hops"] < stats[1]["crit_hops"] // 2
    assert stats[3]["nexport"] < stats[1]["nexport"] // 2
    # auto picks grid blocks for a stencil matrix
    auto = H.tri_plan_stats(H.tri_analyze(L, unit_diag=True, tune=H.tune_default(
        host_only=1, schedule="owner_persistent", num_groups=64)))
    assert auto["crit_hops"] == stats[3]["crit_hops"]
    # an unstructured matrix falls back to contiguous parts
    R = synth.random_lower(3000, 0.002, seed=3)
    a1 = H.tri_plan_stats(H.tri_analyze(R, tune=H.tune_default(host_only=1, schedule="owner_persistent",
                                                               num_groups=16)))
    c1 = H.tri_plan_stats(H.tri_analyze(R, tune=H.tune_default(host_only=1, schedule="owner_persistent",
                                                               num_groups=16, partition=1)))
    assert a1["crit_hops"] == c1["crit_hops"] and a1["nexport"] == c1["nexport"]


def test_queue_parts_read_only_earlier_parts():
    # The queue-mode dataflow kernel needs every part to read only from parts
    # with lower numbers (a part is taken only when all lower ones have been
    # taken by running workgroups); parts never span two independent systems,
    # and the systems with the most levels come first.
    mats = [synth.diffusion2d(30, 21, 1.0, seed=1), synth.diffusion3d(11, 10, 9, 1.0, seed=2),
            synth.poisson2d(7, 3), synth.diffusion3d(14, 13, 12, 1.0, seed=4), synth.poisson2d(45, 2)]
    import scipy.sparse as sp
    m = sp.block_diag([M.to_scipy() for M in mats]).tocsr()
    m.sort_indices()
    A = CSR(m.shape[0], m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())
    sys_ptr = np.cumsum([0] + [M.n for M in mats]).astype(np.int32)
    n = A.n
    t = H.tune_default(host_only=1, max_nrhs=8, part_rows=400, schedule="owner_persistent", kernel_variant=6)
    f = H.batch_setup(A, sys_ptr, "iluk", k=1, tune=t)
    sysof = np.searchsorted(sys_ptr, np.arange(n), side="right") - 1
    for which, plan in enumerate(H.ilu_plans(f)):
        st = H.tri_plan_stats(plan)
        assert st["queue"] == 1 and st["dataflow"] == 1 and st["num_groups"] >= len(mats)
        xperm, owner = H.tri_plan_layout(plan)
        part = np.empty(n, np.int64)
        part[xperm] = owner
        rp, ci, _ = H.ilu_factor(f, which)
        rows = np.repeat(np.arange(n), np.diff(rp))
        off = rows != ci
        assert np.all(part[ci[off]] <= part[rows[off]])
        for g in np.unique(part):
            members = np.flatnonzero(part == g)
            assert len(np.unique(sysof[members])) == 1
            assert len(members) <= 400  # the first cut is an upper bound
            # a contiguous range of the problem order
            assert members.max() - members.min() + 1 == len(members)
        # deepest system first: system 0 (30 x 21 2D grid, 2*21+30-2 levels in ILU(1)... )
        lev_depth = []
        nlev, lp, perm = H.tri_plan_info(plan)
        level = np.empty(n, np.int64)
        for k in range(nlev):
            level[perm[lp[k]:lp[k + 1]]] = k + 1
        depth = [level[sys_ptr[s]:sys_ptr[s + 1]].max() for s in range(len(mats))]
        first_part = [part[sys_ptr[s]:sys_ptr[s + 1]].min() for s in range(len(mats))]
        order = sorted(range(len(mats)), key=lambda s: first_part[s])
        assert [depth[s] for s in order] == sorted(depth, reverse=True)


def test_system_queue_layout():
    # kernel variant 7: whole independent systems per workgroup, each in level
    # order, the longest first; every column is a ring row, a global read
    # (-2 - device row) or padding
    mats = [synth.poisson2d(7, 3), synth.diffusion2d(30, 21, 1.0, seed=1), synth.diffusion3d(9, 8, 7, 1.0, seed=2)]
    import scipy.sparse as sp
    m = sp.block_diag([M.to_scipy() for M in mats]).tocsr()
    m.sort_indices()
    A = CSR(m.shape[0], m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())
    sys_ptr = np.cumsum([0] + [M.n for M in mats]).astype(np.int32)
    t = H.tune_default(host_only=1, max_nrhs=4, schedule="level_persistent", kernel_variant=7)
    f = H.batch_setup(A, sys_ptr, "iluk", k=1, tune=t)
    n = A.n
    sysof = np.searchsorted(sys_ptr, np.arange(n), side="right") - 1
    for which, plan in enumerate(H.ilu_plans(f)):
        st = H.tri_plan_stats(plan)
        assert st["sysq"] == 1 and st["num_groups"] == len(mats)
        xperm, _ = H.tri_plan_layout(plan)
        # device rows: one system after another, each in level order
        s_dev = sysof[xperm]
        runs = [s_dev[0]] + [s_dev[i] for i in range(1, n) if s_dev[i] != s_dev[i - 1]]
        assert len(runs) == len(mats) and sorted(runs) == list(range(len(mats)))
        nlev, lp, perm = H.tri_plan_info(plan)
        level = np.empty(n, np.int64)
        for k in range(nlev):
            level[perm[lp[k]:lp[k + 1]]] = k
        lev_dev = level[xperm]
        for s_ in range(len(mats)):
            idx = np.flatnonzero(s_dev == s_)
            assert np.all(np.diff(lev_dev[idx]) >= 0)
        # the system with the most work comes first (2D 30x21 ILU(1) or 3D 9x8x7)
        assert runs[0] != 0
    with pytest.raises(H.HecError):  # the system queue runs the level schedule only
        H.tri_analyze(synth.random_lower(50, 0.05, seed=1), tune=H.tune_default(
            host_only=1, schedule="owner_persistent", kernel_variant=7))


@pytest.mark.parametrize("nsys,sysq", [(130, 1), (100, 0)])
def test_automatic_system_queue_for_large_batches(nsys, sysq):
    # a batch whose solutions exceed the LDS of all workgroups: with at least
    # half as many systems as compute units (256 assumed without a device) the
    # automatic schedule takes the system queue, with fewer the barrier-free
    # kernel
    import scipy.sparse as sp

    P = synth.poisson2d(90)
    m = sp.block_diag([P.to_scipy()] * nsys).tocsr()
    m.sort_indices()
    A = CSR(m.shape[0], m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())
    ptr = (np.arange(nsys + 1) * P.n).astype(np.int32)
    f = H.batch_setup(A, ptr, "ilu0", tune=H.tune_default(host_only=1, max_nrhs=8))
    st = H.tri_plan_stats(H.ilu_plans(f)[0])
    assert st["sysq"] == sysq and st["syncfree"] == 1 - sysq and st["dataflow"] == 0
