"""GPU parity of the level-scheduled triangular solves (Algorithm 2) against
the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from synth import CSR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1606_00541_amd as H  # noqa: E402
from parity import relerr  # noqa: E402  (normwise and element-wise)

SCHEDS = ["level_launch", "level_persistent", "owner_persistent", "owner_dataflow", "syncfree"]
FP64_TOL = 1e-12


def tune(sched, **kw):
    """Tuning for a schedule name; "owner_dataflow" is the owner schedule run
    by the dataflow kernel (no per-level barrier)."""
    if sched == "owner_dataflow":
        return H.tune_default(schedule="owner_persistent", kernel_variant=4, **kw)
    if sched == "syncfree":  # the barrier-free kernel over the level-ordered layout
        return H.tune_default(schedule="level_launch", kernel_variant=5, **kw)
    if sched == "owner_persistent":  # the LDS-chunked owner kernel (or its generic fallback)
        return H.tune_default(schedule=sched, kernel_variant=2, **kw)
    return H.tune_default(schedule=sched, **kw)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()




def transpose(T):
    m = T.to_scipy().T.tocsr()
    m.sort_indices()
    return CSR(T.n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())


def solve(plan, b, upper=False):
    bt = dev(b)
    xt = torch.empty_like(bt)
    (H.tri_solve_upper if upper else H.tri_solve_lower)(plan, bt, xt)
    torch.cuda.synchronize()
    return xt.cpu().numpy()


@pytest.mark.parametrize("sched", SCHEDS)
def test_config1_poisson64_ilu0(sched):
    A = synth.poisson2d(64)
    L, U = oracle.ilu0(A)
    b = synth.rhs(A.n, 1, 1)
    t = tune(sched)
    pl = H.tri_analyze(L, "lower", unit_diag=True, tune=t)
    pu = H.tri_analyze(U, "upper", tune=t)
    for plan, T, up in ((pl, L, False), (pu, U, True)):
        nlev, lp, perm = H.tri_plan_info(plan)
        lev, nl = oracle.levels(T, upper=up)
        lp2, perm2, _ = oracle.level_schedule(lev, nl, upper=up)
        assert nlev == 127 and np.array_equal(lp, lp2) and np.array_equal(perm, perm2)
    y = solve(pl, b)
    x = solve(pu, y, upper=True)
    yref = oracle.lower_solve(L, b, unit=True)
    xref = oracle.upper_solve(U, yref)
    assert relerr(y, yref) <= FP64_TOL
    assert relerr(x, xref) <= FP64_TOL


def test_schedules_are_bit_identical():
    L = synth.random_lower(5000, 0.0015, seed=21)
    b = synth.rhs(L.n, 2, 22)
    outs = []
    for s in SCHEDS:
        p = H.tri_analyze(L, "lower", tune=tune(s, max_nrhs=2))
        outs.append(solve(p, b))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("upper", [False, True])
@pytest.mark.parametrize("nrhs", [1, 3])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_triangles(sched, upper, nrhs, seed):
    n = 3001 + 17 * seed  # several 64-row tiles and a ragged tail
    L = synth.random_lower(n, 0.002, seed=100 + seed, dense_row=n // 3)
    T = transpose(L) if upper else L
    b = synth.rhs(n, nrhs, 200 + seed)
    # ELL width 1 pushes most entries into the CSR remainder
    for w in (-1, 1):
        p = H.tri_analyze(T, "upper" if upper else "lower", tune=tune(sched, ell_width=w))
        x = solve(p, b, upper)
        ref = (oracle.upper_solve if upper else oracle.lower_solve)(T, b)
        assert relerr(x, ref) <= FP64_TOL


def test_cooperative_lanes_for_long_rows():
    n = 2000
    L = synth.random_lower(n, 0.01, seed=5, dense_row=1500)
    b = synth.rhs(n, 2, 6)
    for sched in ("level_persistent", "owner_persistent"):
        t = tune(sched, group_lanes=8, long_row=4, ell_width=2)
        p = H.tri_analyze(L, "lower", tune=t)
        assert relerr(solve(p, b), oracle.lower_solve(L, b)) <= FP64_TOL


@pytest.mark.parametrize("sched", SCHEDS)
def test_fp32_plans(sched):
    A = synth.diffusion3d(12, 11, 10, 1.0, seed=3)
    L, U = oracle.ilu0(A)
    b = synth.rhs(A.n, 2, 4)
    t = tune(sched)
    pl = H.tri_analyze(oracle.to_f32(L), "lower", unit_diag=True, dtype="f32", tune=t)
    pu = H.tri_analyze(oracle.to_f32(U), "upper", dtype="f32", tune=t)
    ref32 = oracle.upper_solve_f32(oracle.to_f32(U), oracle.lower_solve_f32(oracle.to_f32(L), b, unit=True))
    # FP32 vectors
    y = solve(pl, b.astype(np.float32))
    x = solve(pu, y, upper=True)
    assert x.dtype == np.float32
    assert relerr(x.astype(np.float64), ref32.astype(np.float64)) <= 1e-5
    # FP64 vectors with an FP32 plan: converted on load and store
    y64 = solve(pl, b)
    assert y64.dtype == np.float64
    assert relerr(y64, oracle.lower_solve(L, b, unit=True)) <= 1e-5


def test_empty_and_single_row():
    for n in (0, 1):
        T = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 2.0))
        for s in SCHEDS:
            p = H.tri_analyze(T, "lower", tune=tune(s))
            if n:
                assert np.array_equal(solve(p, np.array([3.0])), np.array([1.5]))


def test_diagonal_and_bidiagonal_closed_forms():
    n = 4097
    D = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 4.0))
    p = H.tri_analyze(D, "lower")
    assert H.tri_plan_info(p)[0] == 1
    b = synth.rhs(n, 1, 9)[:, 0]
    assert np.array_equal(solve(p, b), b / 4.0)
    # unit lower bidiagonal, -1 below: x_i = i (1-based) for b = 1, n levels
    rp = np.concatenate([[0], np.arange(1, 2 * n, 2)]).astype(np.int32)
    ci = np.concatenate([[0]] + [[i - 1, i] for i in range(1, n)]).astype(np.int32)
    v = np.concatenate([[1.0]] + [[-1.0, 1.0] for _ in range(1, n)])
    B = CSR(n, rp, ci, v)
    for s in SCHEDS:
        p = H.tri_analyze(B, "lower", tune=tune(s))
        assert H.tri_plan_info(p)[0] == n
        assert np.array_equal(solve(p, np.ones(n)), np.arange(1, n + 1, dtype=float))


@pytest.mark.parametrize("sched", ["owner_persistent", "owner_dataflow", "syncfree"])
def test_in_place_solve(sched):
    L = synth.random_lower(1500, 0.003, seed=8)
    b = synth.rhs(L.n, 1, 9)[:, 0]
    p = H.tri_analyze(L, "lower", tune=tune(sched))
    bt = dev(b)
    H.tri_solve_lower(p, bt, bt)
    torch.cuda.synchronize()
    assert relerr(bt.cpu().numpy(), oracle.lower_solve(L, b)) <= FP64_TOL


@pytest.mark.parametrize("block,chunk", [(64, 64), (64, 128), (256, 256), (256, 512)])
@pytest.mark.parametrize("nrhs", [1, 3])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_owner_chunked_kernel_bit_identical_to_level_launch(block, chunk, nrhs, dt):
    A = synth.diffusion3d(21, 19, 17, 1.0, seed=12)
    L, U = oracle.iluk(A, 1)
    if dt == "f32":
        L, U = oracle.to_f32(L), oracle.to_f32(U)
    b = synth.rhs(A.n, nrhs, 13).astype(np.float64 if dt == "f64" else np.float32)
    ref_plan_l = H.tri_analyze(L, "lower", unit_diag=True, dtype=dt, tune=H.tune_default(schedule="level_launch"))
    ref_plan_u = H.tri_analyze(U, "upper", dtype=dt, tune=H.tune_default(schedule="level_launch"))
    t = tune("owner_persistent", block_threads=block, chunk_rows=chunk, max_nrhs=nrhs)
    pl = H.tri_analyze(L, "lower", unit_diag=True, dtype=dt, tune=t)
    pu = H.tri_analyze(U, "upper", dtype=dt, tune=t)
    assert H.tri_plan_stats(pl)["nnz_tail"] == 0
    for rep in range(3):  # alternating mailbox halves
        assert np.array_equal(solve(pl, b), solve(ref_plan_l, b))
        assert np.array_equal(solve(pu, b, upper=True), solve(ref_plan_u, b, upper=True))


def test_autotune_returns_a_working_tuning(tmp_path):
    A = synth.poisson3d(24)
    L, U = oracle.ilu0(A)
    cache = str(tmp_path / "tune.jsonl")
    best, us = H.tri_autotune(U, "upper", nrhs=2, cache=cache)
    assert us > 0 and best.schedule in (0, 1, 2, 3) and best.max_nrhs == 2
    p = H.tri_analyze(U, "upper", tune=best)
    b = synth.rhs(A.n, 2, 3)
    assert relerr(solve(p, b, upper=True), oracle.upper_solve(U, b)) <= FP64_TOL
    # the second call finds the problem's signature in the cache
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and '"nrhs": 2' in lines[0]
    best2, us2 = H.tri_autotune(U, "upper", nrhs=2, cache=cache)
    assert best2.as_dict() == best.as_dict() and abs(us2 - us) <= 1e-3 * us
    assert len(open(cache).read().splitlines()) == 1
    # another right-hand-side count is another problem
    H.tri_autotune(U, "upper", nrhs=1, cache=cache, max_seconds=0.5)
    assert len(open(cache).read().splitlines()) == 2


def test_autotune_over_independent_systems():
    mats = [synth.diffusion2d(30, 21, 1.0, seed=31), synth.diffusion3d(11, 10, 9, 1.0, seed=32),
            synth.poisson2d(45, 7)]
    import scipy.sparse as sp
    m = sp.block_diag([Mi.to_scipy() for Mi in mats]).tocsr()
    m.sort_indices()
    A = CSR(m.shape[0], m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.copy())
    sys_ptr = np.cumsum([0] + [Mi.n for Mi in mats]).astype(np.int32)
    L, _ = oracle.iluk(A, 1)
    best, us = H.tri_autotune(L, "lower", unit_diag=True, dtype="f32", nrhs=4, sys_ptr=sys_ptr)
    assert us > 0
    f = H.batch_setup(A, sys_ptr, "iluk", k=1, factor_dtype="f32", tune=best)
    r = synth.rhs(A.n, 4, 33)
    rt = dev(r)
    zt = torch.empty_like(rt)
    H.ilu_apply(f, rt, zt)
    torch.cuda.synchronize()
    L, U = oracle.iluk(A, 1)
    assert relerr(zt.cpu().numpy(), oracle.ilu_apply_f32(oracle.to_f32(L), oracle.to_f32(U), r)) <= 1e-5


def test_mailbox_recovers_across_rhs_widths():
    # a plan used with growing then shrinking RHS counts keeps its mailbox
    # halves consistent (resets cover the widest layout ever allocated)
    A = synth.poisson3d(20)
    L, _ = oracle.ilu0(A)
    for sched in ("level_persistent", "owner_persistent", "owner_dataflow"):
        p = H.tri_analyze(L, "lower", unit_diag=True, tune=tune(sched, max_nrhs=4))
        for R in (1, 4, 1, 2, 4, 1):
            b = synth.rhs(A.n, R, R)
            assert relerr(solve(p, b), oracle.lower_solve(L, b, unit=True)) <= FP64_TOL


@pytest.mark.parametrize("groups", [0, 7, 64])
@pytest.mark.parametrize("nrhs", [1, 3])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("part", [1, 3])
def test_dataflow_kernel_bit_identical_to_level_launch(groups, nrhs, dt, part):
    A = synth.diffusion3d(21, 19, 17, 1.0, seed=12)
    L, U = oracle.iluk(A, 1)
    if dt == "f32":
        L, U = oracle.to_f32(L), oracle.to_f32(U)
    b = synth.rhs(A.n, nrhs, 13).astype(np.float64 if dt == "f64" else np.float32)
    ref_l = H.tri_analyze(L, "lower", unit_diag=True, dtype=dt, tune=H.tune_default(schedule="level_launch"))
    ref_u = H.tri_analyze(U, "upper", dtype=dt, tune=H.tune_default(schedule="level_launch"))
    t = tune("owner_dataflow", num_groups=groups, max_nrhs=nrhs, partition=part)
    pl = H.tri_analyze(L, "lower", unit_diag=True, dtype=dt, tune=t)
    pu = H.tri_analyze(U, "upper", dtype=dt, tune=t)
    for rep in range(3):  # alternating mailbox halves
        assert np.array_equal(solve(pl, b), solve(ref_l, b))
        assert np.array_equal(solve(pu, b, upper=True), solve(ref_u, b, upper=True))


def test_dataflow_kernel_with_csr_tails():
    # ILUT rows overflow a narrow ELL part into the CSR remainder
    A = synth.diffusion3d(14, 13, 12, 2.0, seed=5)
    L, U = oracle.ilut(A, 10, 1e-3)
    b = synth.rhs(A.n, 2, 6)
    for T, up, unit in ((L, False, True), (U, True, False)):
        ref = H.tri_analyze(T, "upper" if up else "lower", unit_diag=unit,
                            tune=H.tune_default(schedule="level_launch", ell_width=2))
        p = H.tri_analyze(T, "upper" if up else "lower", unit_diag=unit,
                          tune=tune("owner_dataflow", ell_width=2, max_nrhs=2))
        assert H.tri_plan_stats(p)["nnz_tail"] > 0
        assert np.array_equal(solve(p, b, up), solve(ref, b, up))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("nrhs", [1, 2])
def test_dataflow_wide_rows_bit_identical(dt, nrhs):
    # ILUT rows of up to 12 entries: the dataflow kernel's automatic width
    # covers the longest row (widths 10, 12 or 16), so no CSR tail is left
    A = synth.diffusion3d(13, 12, 11, 2.0, seed=8)
    L, U = oracle.ilut(A, 12, 1e-4)
    if dt == "f32":
        L, U = oracle.to_f32(L), oracle.to_f32(U)
    b = synth.rhs(A.n, nrhs, 9).astype(np.float64 if dt == "f64" else np.float32)
    for T, up, unit in ((L, False, True), (U, True, False)):
        uplo = "upper" if up else "lower"
        ref = H.tri_analyze(T, uplo, unit_diag=unit, dtype=dt, tune=H.tune_default(schedule="level_launch"))
        p = H.tri_analyze(T, uplo, unit_diag=unit, dtype=dt, tune=tune("owner_dataflow", max_nrhs=nrhs))
        st = H.tri_plan_stats(p)
        assert st["ell_width"] in (10, 12, 16) and st["nnz_tail"] == 0 and st["dataflow"] == 1
        for rep in range(2):
            assert np.array_equal(solve(p, b, up), solve(ref, b, up))


@pytest.mark.parametrize("nrhs", [1, 5])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_syncfree_bit_identical_to_level_launch_with_tails(nrhs, dt):
    # ILU(1) factors with ELL width 2 (most entries in CSR tails), many levels
    A = synth.diffusion3d(14, 12, 11, 1.5, seed=17)
    L, U = oracle.iluk(A, 1)
    b = synth.rhs(A.n, nrhs, 18)
    for T, up in ((L, False), (U, True)):
        uplo = "upper" if up else "lower"
        outs = []
        for s in ("level_launch", "syncfree"):
            p = H.tri_analyze(T, uplo, unit_diag=not up, dtype=dt, tune=tune(s, ell_width=2, max_nrhs=nrhs))
            bt = dev(b if dt == "f64" else b.astype(np.float32))
            xt = torch.empty_like(bt)
            (H.tri_solve_upper if up else H.tri_solve_lower)(p, bt, xt)
            outs.append(xt.cpu().numpy())
        assert np.array_equal(outs[0], outs[1])
