"""GPU parity of the ILU, RAS and batched preconditioners (Section 3,
eq. (1) and eq. (4)), the Krylov solvers and graph replay, against the CPU
oracle."""
import numpy as np
import pytest

import oracle
import synth
from synth import CSR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1606_00541_amd as H  # noqa: E402
from parity import relerr  # noqa: E402  (normwise and element-wise)

FP64_TOL = 1e-12


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()




def apply(f, r):
    rt = dev(r)
    zt = torch.empty_like(rt)
    (H.ras_apply if isinstance(f, H.Ras) else H.ilu_apply)(f, rt, zt)
    torch.cuda.synchronize()
    return zt.cpu().numpy()


def same_csr(rp, ci, v, T):
    return np.array_equal(rp, T.rowptr) and np.array_equal(ci, T.col) and np.array_equal(v, T.val)


@pytest.mark.parametrize("sched", ["level_persistent", "owner_persistent"])
def test_config2_poisson128_ilu0_full_size(sched):
    A = synth.poisson3d(128)
    f = H.ilu_setup(A, "ilu0", tune=H.tune_default(schedule=sched))
    L, U = oracle.ilu0(A)
    assert same_csr(*H.ilu_factor(f, 0), L) and same_csr(*H.ilu_factor(f, 1), U)
    pl, pu = H.ilu_plans(f)
    assert H.tri_plan_info(pl)[0] == 382 and H.tri_plan_info(pu)[0] == 382
    st = H.tri_plan_stats(pl)
    assert st["ell_width"] == 3 and st["nnz_tail"] == 0
    r = synth.rhs(A.n, 1, 2)
    z = apply(f, r)
    assert relerr(z, oracle.ilu_apply(L, U, r)) <= FP64_TOL


@pytest.mark.parametrize("kind,args", [("ilu0", {}), ("iluk", {"k": 1}), ("iluk", {"k": 2}),
                                       ("ilut", {"p": 10, "tol": 1e-3})])
def test_ilu_kinds_match_oracle(kind, args):
    A = synth.diffusion3d(14, 13, 12, 2.0, seed=3)
    f = H.ilu_setup(A, kind, tune=H.tune_default(max_nrhs=4), **args)
    if kind == "ilu0":
        L, U = oracle.ilu0(A)
    elif kind == "iluk":
        L, U = oracle.iluk(A, args["k"])
    else:
        L, U = oracle.ilut(A, args["p"], args["tol"])
    assert same_csr(*H.ilu_factor(f, 0), L) and same_csr(*H.ilu_factor(f, 1), U)
    r = synth.rhs(A.n, 4, 5)
    assert relerr(apply(f, r), oracle.ilu_apply(L, U, r)) <= FP64_TOL


def test_fp32_factors_fp64_vectors():
    A = synth.diffusion3d(16, 16, 16, 2.0, seed=3)
    f = H.ilu_setup(A, "ilut", p=10, tol=1e-3, factor_dtype="f32")
    L, U = oracle.ilut(A, 10, 1e-3)
    r = synth.rhs(A.n, 1, 3)
    ref = oracle.ilu_apply_f32(oracle.to_f32(L), oracle.to_f32(U), r)
    z = apply(f, r)
    assert z.dtype == np.float64
    assert relerr(z, ref) <= 1e-5
    assert relerr(z, oracle.ilu_apply(L, U, r)) <= 1e-4


@pytest.mark.parametrize("fdt", ["f64", "f32"])
def test_ras_matches_oracle(fdt):
    A = synth.poisson3d(18)
    owner, _ = synth.subdomain_cuts(A.n, 6, 500, 1500, seed=4)
    s = H.ras_setup(A, 6, owner, overlap=1, factor_dtype=fdt, tune=H.tune_default(max_nrhs=3))
    doms = oracle.ras_setup(A, owner, 6, overlap=1)
    nsub, tot, sizes = H.ras_info(s)
    assert nsub == 6 and list(sizes) == [len(d.ext) for d in doms]
    r = synth.rhs(A.n, 3, 5)
    z = apply(s, r)
    if fdt == "f64":
        assert relerr(z, oracle.ras_apply(doms, r)) <= FP64_TOL
    else:
        assert relerr(z, oracle.ras_apply_f32(oracle.ras_to_f32(doms), r)) <= 1e-5



@pytest.mark.parametrize("fdt", ["f64", "f32"])
@pytest.mark.parametrize("overlap", [0, 1])
@pytest.mark.parametrize("kind,args", [("iluk", {"k": 1}), ("ilut", {"p": 7, "tol": 0.1}),
                                       ("ilut", {"p": 10, "tol": 1e-3})])
def test_block_ilu_and_ras_ilu_match_oracle(kind, args, overlap, fdt):
    # BILU(k) / BILUT (overlap 0) and RAS with ILU(k) / ILUT subdomains
    A = synth.diffusion3d(16, 14, 12, 1.0, seed=9)
    owner = synth.grid_bisection(16, 14, 12, 8)
    s = H.ras_setup_ilu(A, 8, owner, overlap=overlap, kind=kind, factor_dtype=fdt,
                        tune=H.tune_default(max_nrhs=2), **args)
    oargs = {"k": args["k"]} if kind == "iluk" else {"p": args["p"], "tau": args["tol"]}
    doms = oracle.ras_setup(A, owner, 8, overlap=overlap, kind=kind, **oargs)
    assert list(H.ras_info(s)[2]) == [len(d.ext) for d in doms]
    r = synth.rhs(A.n, 2, 6)
    z = apply(s, r)
    if fdt == "f64":
        assert relerr(z, oracle.ras_apply(doms, r)) <= FP64_TOL
    else:
        assert relerr(z, oracle.ras_apply_f32(oracle.ras_to_f32(doms), r)) <= 1e-5


def test_gmres20_with_block_ilut():
    # the paper's solver and block preconditioner pairing (Section 4, GMRES(20))
    A = synth.poisson3d(24)
    owner = synth.grid_bisection(24, 24, 24, 16)
    s = H.ras_setup_ilu(A, 16, owner, overlap=0, kind="ilut", p=7, tol=0.1)
    M = H.hec_from_csr(A)
    b = synth.rhs(A.n, 1, 1)
    xt = torch.zeros(A.n, 1, dtype=torch.float64, device="cuda")
    st, info = H.krylov_solve(M, s, dev(b), xt, method="gmres", m=20, rtol=1e-10)
    assert st == 0 and info[0].relres <= 1e-10
    x = xt.cpu().numpy()[:, 0]
    assert np.linalg.norm(b[:, 0] - oracle.spmv(A, x)) / np.linalg.norm(b[:, 0]) <= 1e-10
    doms = oracle.ras_setup(A, owner, 16, overlap=0, kind="ilut", p=7, tau=0.1)
    xo, oinfo = oracle.fgmres(A, b[:, 0], lambda v: oracle.ras_apply(doms, v), m=20, rtol=1e-10)
    assert oinfo.converged and abs(info[0].iters - oinfo.iters) <= 2


def _block_diag(mats):
    rps, cis, vs, sys_ptr, off, nnz = [np.zeros(1, np.int64)], [], [], [0], 0, 0
    for M in mats:
        rps.append(M.rowptr[1:].astype(np.int64) + nnz)
        cis.append(M.col.astype(np.int64) + off)
        vs.append(M.val)
        off += M.n
        nnz += M.nnz
        sys_ptr.append(off)
    return CSR(off, np.concatenate(rps).astype(np.int32), np.concatenate(cis).astype(np.int32),
               np.concatenate(vs)), np.array(sys_ptr, np.int32)


def test_batch_matches_per_system_oracle():
    mats = [synth.diffusion2d(30, 20, 1.0, seed=1), synth.diffusion3d(9, 8, 7, 1.0, seed=2),
            synth.poisson2d(5, 3), synth.diffusion3d(13, 13, 13, 1.0, seed=4), synth.poisson2d(41, 1)]
    A, sys_ptr = _block_diag(mats)
    f = H.batch_setup(A, sys_ptr, "iluk", k=1, tune=H.tune_default(max_nrhs=8))
    r = synth.rhs(A.n, 8, 7)
    z = apply(f, r)
    for s, M in enumerate(mats):
        L, U = oracle.iluk(M, 1)
        seg = slice(int(sys_ptr[s]), int(sys_ptr[s + 1]))
        assert relerr(z[seg], oracle.ilu_apply(L, U, r[seg])) <= FP64_TOL


def test_batch_and_ras_on_the_barrier_free_kernel():
    # many independent systems / subdomains solved in one barrier-free launch
    mats = [synth.diffusion2d(15 + 3 * i, 11, 1.0, seed=60 + i) for i in range(5)]
    A, sys_ptr = _block_diag(mats)
    t = H.tune_default(schedule="level_launch", kernel_variant=5, max_nrhs=3)
    f = H.batch_setup(A, sys_ptr, "iluk", k=1, tune=t)
    g = H.batch_setup(A, sys_ptr, "iluk", k=1, tune=H.tune_default(schedule="level_launch", max_nrhs=3))
    r = synth.rhs(A.n, 3, 61)
    assert np.array_equal(apply(f, r), apply(g, r))
    B = synth.poisson3d(16)
    owner, _ = synth.subdomain_cuts(B.n, 6, 400, 1000, seed=62)
    s1 = H.ras_setup(B, 6, owner, overlap=1, factor_dtype="f32", tune=t)
    s2 = H.ras_setup(B, 6, owner, overlap=1, factor_dtype="f32",
                     tune=H.tune_default(schedule="level_launch", max_nrhs=3))
    r = synth.rhs(B.n, 3, 63)
    assert np.array_equal(apply(s1, r), apply(s2, r))


def test_batch_rejects_coupled_systems():
    A = synth.poisson2d(6)
    with pytest.raises(H.HecError) as e:
        H.batch_setup(A, np.array([0, 18, 36], np.int32))
    assert e.value.name == "INVALID_ARG"


def test_hec_matrix_roundtrip_and_spmv():
    A = synth.diffusion3d(10, 9, 8, 1.5, seed=6)
    M = H.hec_from_csr(A, ell_width=4)
    h = H.hec_matrix_export(M)
    T = oracle.hec_to_csr(A.n, h["width"], h["ld"], h["ell_col"], h["ell_val"], h["csr_ptr"], h["csr_col"],
                          h["csr_val"])
    assert np.array_equal(T.rowptr, A.rowptr) and np.array_equal(T.col, A.col) and np.array_equal(T.val, A.val)
    x = synth.rhs(A.n, 2, 8)
    xt = dev(x)
    yt = torch.empty_like(xt)
    H.hec_spmv(M, xt, yt)
    torch.cuda.synchronize()
    assert relerr(yt.cpu().numpy(), oracle.spmv(A, x)) <= 1e-14


def test_gmres_ilu0_reaches_tolerance():
    A = synth.poisson3d(24)
    f = H.ilu_setup(A, "ilu0")
    M = H.hec_from_csr(A)
    b = synth.rhs(A.n, 2, 2)
    xt = torch.zeros(A.n, 2, dtype=torch.float64, device="cuda")
    st, info = H.krylov_solve(M, f, dev(b), xt, method="gmres", m=30, rtol=1e-10)
    x = xt.cpu().numpy()
    assert st == 0
    L, U = oracle.ilu0(A)
    for k in range(2):
        true = np.linalg.norm(b[:, k] - oracle.spmv(A, x[:, k])) / np.linalg.norm(b[:, k])
        assert true <= 1e-10 and abs(true - info[k].relres) <= 1e-12
        xo, io = oracle.fgmres(A, b[:, k], lambda v: oracle.ilu_apply(L, U, v), m=30, rtol=1e-10)
        assert relerr(x[:, k], xo) <= 1e-7
        assert abs(info[k].iters - io.iters) <= 2


def test_fgmres_mixed_precision_refinement():
    A = synth.diffusion3d(16, 16, 16, 2.0, seed=3)
    f32 = H.ilu_setup(A, "ilut", p=10, tol=1e-3, factor_dtype="f32")
    M = H.hec_from_csr(A)
    b = synth.rhs(A.n, 1, 3)
    xt = torch.zeros(A.n, 1, dtype=torch.float64, device="cuda")
    st, info = H.krylov_solve(M, f32, dev(b), xt, method="fgmres", m=30, rtol=1e-10)
    assert st == 0
    x = xt.cpu().numpy()[:, 0]
    true = np.linalg.norm(b[:, 0] - oracle.spmv(A, x)) / np.linalg.norm(b[:, 0])
    assert true <= 1e-10
    L, U = oracle.ilut(A, 10, 1e-3)
    xo, _ = oracle.fgmres(A, b[:, 0], lambda v: oracle.ilu_apply(L, U, v), m=30, rtol=1e-10)
    assert relerr(x, xo) <= 1e-6


def test_bicgstab_ras_fp32_multi_rhs():
    A = synth.poisson3d(20)
    owner, _ = synth.subdomain_cuts(A.n, 8, 600, 1600, seed=4)
    s = H.ras_setup(A, 8, owner, overlap=1, factor_dtype="f32", tune=H.tune_default(max_nrhs=4))
    M = H.hec_from_csr(A)
    b = synth.rhs(A.n, 4, 4)
    xt = torch.zeros(A.n, 4, dtype=torch.float64, device="cuda")
    st, info = H.krylov_solve(M, s, dev(b), xt, method="bicgstab", rtol=1e-10)
    assert st == 0
    x = xt.cpu().numpy()
    for k in range(4):
        true = np.linalg.norm(b[:, k] - oracle.spmv(A, x[:, k])) / np.linalg.norm(b[:, k])
        assert true <= 1e-10


def test_krylov_reports_not_converged():
    A = synth.poisson3d(12)
    f = H.ilu_setup(A, "ilu0")
    M = H.hec_from_csr(A)
    b = synth.rhs(A.n, 1, 1)
    xt = torch.zeros(A.n, 1, dtype=torch.float64, device="cuda")
    st, info = H.krylov_solve(M, f, dev(b), xt, method="gmres", m=5, rtol=1e-10, maxit=2)
    assert st == 8 and info[0].status == 8 and info[0].iters == 2


@pytest.mark.parametrize("kind", ["ilu", "ras"])
def test_graph_replay_matches_eager(kind):
    A = synth.poisson3d(16)
    if kind == "ilu":
        M = H.ilu_setup(A, "ilu0", tune=H.tune_default(schedule="owner_persistent", max_nrhs=2))
    else:
        owner, _ = synth.subdomain_cuts(A.n, 4, 600, 1500, seed=2)
        M = H.ras_setup(A, 4, owner, overlap=1, factor_dtype="f32", tune=H.tune_default(max_nrhs=2))
    r = dev(synth.rhs(A.n, 2, 3))
    z = torch.empty_like(r)
    g = H.hec_graph_capture(M, r, z)
    ze = torch.empty_like(r)
    for rep in range(4):
        r.mul_(0.5).add_(float(rep))  # eager work between replays changes the input
        H.hec_graph_launch(g)
        torch.cuda.synchronize()
        got = z.clone()
        (H.ras_apply if kind == "ras" else H.ilu_apply)(M, r, ze)
        torch.cuda.synchronize()
        assert torch.equal(got, ze)


@pytest.mark.parametrize("kernel", ["auto", "syncfree"])
@pytest.mark.parametrize("method", ["fgmres", "bicgstab"])
@pytest.mark.parametrize("fdt", ["f64", "f32"])
def test_batch_krylov_solves_each_system_alone(method, fdt, kernel):
    # every (system, rhs) pair is its own Krylov problem: the result and the
    # iteration count match the oracle solving that system by itself
    mats = [synth.diffusion2d(30, 20, 1.0, seed=1), synth.diffusion3d(9, 8, 7, 1.0, seed=2),
            synth.poisson2d(5, 3), synth.diffusion3d(13, 13, 13, 1.0, seed=4), synth.poisson2d(41, 1)]
    A, sys_ptr = _block_diag(mats)
    R = 2
    # the barrier-free kernel skips the rows of problems that have finished
    kw = {"schedule": "level_launch", "kernel_variant": 5} if kernel == "syncfree" else {}
    f = H.batch_setup(A, sys_ptr, "iluk", k=1, factor_dtype=fdt, tune=H.tune_default(max_nrhs=R, **kw))
    M = H.hec_from_csr(A)
    b = synth.rhs(A.n, R, 11)
    b[int(sys_ptr[2]):int(sys_ptr[3]), 1] = 0.0  # a zero right-hand side: x = 0 for that pair
    xt = torch.zeros(A.n, R, dtype=torch.float64, device="cuda")
    st, info = H.krylov_solve_batch(M, f, sys_ptr, dev(b), xt, method=method, m=30, rtol=1e-10)
    assert st == 0 and len(info) == len(mats) * R
    x = xt.cpu().numpy()
    for s, Ms in enumerate(mats):
        seg = slice(int(sys_ptr[s]), int(sys_ptr[s + 1]))
        L, U = oracle.iluk(Ms, 1)
        if fdt == "f32":
            L32, U32 = oracle.to_f32(L), oracle.to_f32(U)
            prec = lambda v: oracle.ilu_apply_f32(L32, U32, v)  # noqa: E731
        else:
            prec = lambda v: oracle.ilu_apply(L, U, v)  # noqa: E731
        for k in range(R):
            q = info[s * R + k]
            bs = b[seg, k]
            if not np.any(bs):
                assert np.all(x[seg, k] == 0.0) and q.iters == 0
                continue
            true = np.linalg.norm(bs - oracle.spmv(Ms, x[seg, k])) / np.linalg.norm(bs)
            assert true <= 1e-10 and abs(true - q.relres) <= 1e-12
            solver = oracle.fgmres if method == "fgmres" else oracle.bicgstab
            kw = {"m": 30} if method == "fgmres" else {}
            xo, io = solver(Ms, bs, prec, rtol=1e-10, **kw)
            assert relerr(x[seg, k], xo) <= 1e-7
            assert abs(q.iters - io.iters) <= (2 if method == "fgmres" else 5)


def test_batch_krylov_rejects_coupling():
    A = synth.poisson2d(6)
    M = H.hec_from_csr(A)
    b = dev(synth.rhs(A.n, 1, 1))
    x = torch.zeros_like(b)
    with pytest.raises(H.HecError) as e:
        H.krylov_solve_batch(M, None, np.array([0, 18, 36], np.int32), b, x)
    assert e.value.name == "INVALID_ARG"


@pytest.mark.parametrize("fdt", ["f64", "f32"])
@pytest.mark.parametrize("R", [1, 4, 8, 16])
def test_system_queue_matches_level_launches(fdt, R):
    # kernel variant 7 computes every row as the per-level launches do: the
    # same bits, for batches (systems) and RAS (subdomains)
    mats = [synth.diffusion2d(60, 41, 1.0, seed=41), synth.diffusion3d(13, 12, 11, 1.0, seed=42),
            synth.poisson2d(5, 3), synth.diffusion3d(17, 16, 15, 1.0, seed=44), synth.poisson2d(90, 4)]
    A, sys_ptr = _block_diag(mats)
    tq = H.tune_default(schedule="level_persistent", kernel_variant=7, max_nrhs=R, block_threads=512)
    tl = H.tune_default(schedule="level_launch", max_nrhs=R)
    f = H.batch_setup(A, sys_ptr, "iluk", k=1, factor_dtype=fdt, tune=tq)
    g = H.batch_setup(A, sys_ptr, "iluk", k=1, factor_dtype=fdt, tune=tl)
    assert H.tri_plan_stats(H.ilu_plans(f)[0])["sysq"] == 1
    r = synth.rhs(A.n, R, 45)
    for rep in range(2):  # the queue counter resets between launches
        assert np.array_equal(apply(f, r), apply(g, r))
    B = synth.poisson3d(24)
    owner, _ = synth.subdomain_cuts(B.n, 8, 1000, 2500, seed=46)
    s1 = H.ras_setup(B, 8, owner, overlap=1, factor_dtype=fdt, tune=tq)
    s2 = H.ras_setup(B, 8, owner, overlap=1, factor_dtype=fdt, tune=tl)
    r = synth.rhs(B.n, R, 47)
    assert np.array_equal(apply(s1, r), apply(s2, r))
    doms = oracle.ras_setup(B, owner, 8, overlap=1)
    ref = oracle.ras_apply(doms, r) if fdt == "f64" else oracle.ras_apply_f32(oracle.ras_to_f32(doms), r)
    assert relerr(apply(s1, r), ref) <= (FP64_TOL if fdt == "f64" else 1e-5)


@pytest.mark.parametrize("fdt", ["f64", "f32"])
def test_system_queue_wide_levels(fdt):
    # 16 right-hand sides in two groups of 8 per row: levels of up to 520
    # rows give 1040 items, more than the 512 threads hold in flight twice,
    # so the widest levels also take the direct path
    A = synth.poisson2d(520)
    R = 16
    tq = H.tune_default(schedule="level_persistent", kernel_variant=7, max_nrhs=R, block_threads=512)
    tl = H.tune_default(schedule="level_launch", max_nrhs=R)
    f = H.ilu_setup(A, "ilu0", factor_dtype=fdt, tune=tq)
    g = H.ilu_setup(A, "ilu0", factor_dtype=fdt, tune=tl)
    st = H.tri_plan_stats(H.ilu_plans(f)[0])
    assert st["sysq"] == 1
    r = synth.rhs(A.n, R, 49)
    z = apply(f, r)
    assert np.array_equal(z, apply(g, r))
    L, U = oracle.ilu0(A)
    if fdt == "f64":
        assert relerr(z, oracle.ilu_apply(L, U, r)) <= FP64_TOL
    else:
        assert relerr(z, oracle.ilu_apply_f32(oracle.to_f32(L), oracle.to_f32(U), r)) <= 1e-5


def test_system_queue_reads_beyond_its_ring():
    # 64 right-hand sides of a wide-level system: the ring holds one level at
    # most, so every dependency is read back from the workspace
    A = synth.poisson2d(300)
    t = H.tune_default(schedule="level_persistent", kernel_variant=7, max_nrhs=64, block_threads=1024)
    f = H.ilu_setup(A, "ilu0", tune=t)
    g = H.ilu_setup(A, "ilu0", tune=H.tune_default(schedule="level_launch", max_nrhs=64))
    r = synth.rhs(A.n, 64, 48)
    z = apply(f, r)
    assert np.array_equal(z, apply(g, r))
    L, U = oracle.ilu0(A)
    assert relerr(z, oracle.ilu_apply(L, U, r)) <= FP64_TOL


@pytest.mark.parametrize("R", [1, 3, 4])
def test_gmres_both_orthogonalizations_match_oracle(R):
    # R = 1, 4: the re-orthogonalization delayed into the next step; R = 3:
    # two classical passes per step.  A short restart length takes several
    # cycles, each closed by the extra inner-product pass of the delayed form.
    A = synth.poisson3d(14)
    f = H.ilu_setup(A, "ilu0", tune=H.tune_default(max_nrhs=R))
    M = H.hec_from_csr(A)
    b = synth.rhs(A.n, R, 21)
    xt = torch.zeros(A.n, R, dtype=torch.float64, device="cuda")
    st, info = H.krylov_solve(M, f, dev(b), xt, method="gmres", m=4, rtol=1e-10)
    assert st == 0
    x = xt.cpu().numpy()
    L, U = oracle.ilu0(A)
    for k in range(R):
        xo, io = oracle.fgmres(A, b[:, k], lambda v: oracle.ilu_apply(L, U, v), m=4, rtol=1e-10)
        assert relerr(x[:, k], xo) <= 1e-7
        assert abs(info[k].iters - io.iters) <= 2 and info[k].restarts >= 2
        assert info[k].precond_applies in (info[k].iters, info[k].iters + 1)
    # the iteration limit reached in the middle of a cycle
    xt.zero_()
    st, info = H.krylov_solve(M, f, dev(b), xt, method="gmres", m=4, rtol=1e-14, maxit=6)
    assert st == 8 and all(q.status == 8 and q.iters == 6 for q in info)
