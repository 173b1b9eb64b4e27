"""Benchmark of the level-scheduled L+U solve path on one MI355X.

Workload (default): 3D 7-point Poisson on a 128^3 grid (n = 2,097,152, natural
ordering, 382 levels per triangle), ILU(0) factors in FP64 stored as HEC with
ELL width 3 per triangle, one right-hand side U[-1,1] (seed 2).  One step is
one preconditioner application z = (LU)^{-1} r: the gather of r into level
order, the level-scheduled L solve, the map into U's order, the U solve and
the scatter of z (eq. (1), Algorithm 2).  Inputs are resident in HBM before
timing starts.  The same factors then drive restarted GMRES(30) to a true
relative residual of 1e-10, timed as a whole solve.

value = counted L+U bytes per application / time per application (GB/s);
counted bytes = off-diagonal values and column indices of L and U, U's
diagonal, the two level permutations, and per RHS one read and one write of
each of b, y, x (y twice); ELL padding excluded.

The CPU baseline is the test oracle (serial C substitution on CSR, natural
order) timed on a bounded number of full L+U applications of the same system.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def counted_bytes(n, nnz_l, nnz_u, nrhs, sv=8, unit_l=True):
    """Algorithmic bytes of one L+U application (see module docstring)."""
    diag = n * sv * (1 if unit_l else 2)
    return (nnz_l + nnz_u) * (sv + 4) + diag + 2 * 4 * n + nrhs * 4 * n * sv


def per_launch_bytes(n, nnz, nrhs, sv=8, diag=False):
    """Algorithmic bytes of one triangular-solve launch: values + indices,
    the diagonal if stored, one permutation, read b and write x per RHS."""
    return nnz * (sv + 4) + (n * sv if diag else 0) + 4 * n + nrhs * 2 * n * sv


def kernel_source_hash():
    """Short hash of the triangular-solve kernel sources (to tie counter
    readings to the code they were taken on)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("tri_kernels.hip", "hec_dev.h"):
        with open(os.path.join(ROOT, "paper_1606_00541_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summaries
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None
    when no summary matches the current kernel sources."""
    src = kernel_source_hash()
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for fn in sorted(os.listdir(pdir)):
        if not fn.endswith(".md"):
            continue
        for line in open(os.path.join(pdir, fn)):
            if not line.startswith("TRAFFIC "):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("src") == src:
                return 1024.0 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                                 float(kv["write_kib"]) * float(kv["write_scale"]))
    return None


def _rep_stats(H, torch, f, r, z, stream, reps, cold):
    """Median and p10/p90 of single L+U applications, each bracketed by its
    own HIP events on the launch stream.  Cold: a 512 MiB buffer is rewritten
    before every application so that neither L2 nor the Infinity Cache holds
    the factors (the fill itself lies outside the events)."""
    import numpy as np

    flush = torch.empty((512 << 20) // 8, dtype=torch.float64, device="cuda") if cold else None
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for i, (a, b) in enumerate(ev):
        if cold:
            flush.fill_(float(i))
        a.record(stream)
        H.ilu_apply(f, r, z)
        b.record(stream)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"reps": reps, "median": round(float(np.median(t)), 5), "p10": round(float(np.percentile(t, 10)), 5),
            "p90": round(float(np.percentile(t, 90)), 5)}


def _extras(H, torch, np, f, A, r, z, stream, args):
    """Device refactorization timing (same values: the applications after it
    must not change) and the per-application warm / cold spreads."""
    z_before = z.clone()
    av = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).cuda()
    t0 = time.time()
    H.ilu_refactor(f, A, av)
    refac_first = time.time() - t0
    t0 = time.time()
    for _ in range(5):
        H.ilu_refactor(f, None, av)
    refac = (time.time() - t0) / 5
    H.ilu_apply(f, r, z)
    torch.cuda.synchronize()
    refac_same = bool(torch.equal(z, z_before))
    reps = _rep_stats(H, torch, f, r, z, stream, args.steps, cold=False)
    reps_cold = _rep_stats(H, torch, f, r, z, stream, min(args.steps, 20), cold=True)
    return refac, refac_first, refac_same, reps, reps_cold


def _time_apply(H, torch, f, r, z, steps, warmup, ras=False):
    app = H.ras_apply if ras else H.ilu_apply
    for _ in range(warmup):
        app(f, r, z)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        app(f, r, z)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _krylov(H, torch, M, Aop, b, method, rtol=1e-10, maxit=20000):
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.time()
    st, info = H.krylov_solve(Aop, M, b, x, method=method, m=30, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    dt = time.time() - t0
    return x, {"status": int(st), "seconds": round(dt, 4), "iters": [i.iters for i in info],
               "precond_applies": [i.precond_applies for i in info],
               "relres_max": max(i.relres for i in info)}


def _krylov_batch(H, torch, M, Aop, sys_ptr, b, method, rtol=1e-10, maxit=20000):
    """Each (system, rhs) pair as its own Krylov problem (krylov_solve_batch)."""
    import numpy as np

    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.time()
    st, info = H.krylov_solve_batch(Aop, M, sys_ptr, b, x, method=method, m=30, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    dt = time.time() - t0
    its = np.array([i.iters for i in info])
    return x, {"status": int(st), "seconds": round(dt, 4), "problems": len(info),
               "iters_max": int(its.max()), "iters_median": float(np.median(its)), "iters_min": int(its.min()),
               "relres_max": max(i.relres for i in info)}


def _block_diag(mats):
    import numpy as np

    from synth import CSR
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


def _log(msg):
    """Progress to stderr (the JSON line alone goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _tune(H, args, **kw):
    sched = 0 if args.schedule == "auto" else args.schedule
    if args.block_threads:
        kw.setdefault("block_threads", args.block_threads)
    return H.tune_default(schedule=sched, kernel_variant=args.kernel_variant, **kw)


def _kernel_name(st):
    """The kernel a plan runs (from tri_plan_stats)."""
    if st["dataflow"]:
        return "k_dataflow" + (" (part queue)" if st.get("queue") else "")
    if st["syncfree"]:
        return "k_syncfree"
    if st["sysq"]:
        # the pipelined system queue: no CSR tail, ELL width 1..8, RHS in
        # groups of 4 or 8; otherwise the plain system queue
        R = st.get("nrhs", 0)
        ok = st["nnz_tail"] == 0 and 1 <= st["ell_width"] <= 8 and R % 4 == 0
        return "k_sysq_pipe" if ok else "k_sysq"
    return "k_level" if st["schedule"] == 1 else "k_persistent"


def _roofline(st, bytes_per_apply, ms):
    """Roofline of the dominant kernel: the L and U launches share it, so its
    average launch moves half the counted bytes in half the application."""
    launches = st["nlev"] * 2 if (st["schedule"] == 1 and not st["syncfree"]) else 2
    per_launch = bytes_per_apply / launches
    achieved = per_launch / (ms / launches * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": _kernel_name(st), "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "algorithmic_bytes_per_launch": int(per_launch), "traffic": None}


def _graph_ms(H, torch, M, r, z, reps):
    """One application replayed from a captured HIP graph (hec_graph_capture)."""
    g = H.hec_graph_capture(M, r, z)
    for _ in range(2):
        H.hec_graph_launch(g)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        H.hec_graph_launch(g)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


_NATIVE = {}


def _native_oracle():
    """Switch the oracle to a -O3 -march=native build made on this host (the
    CPU baseline's build; same arithmetic as the test build).  Returns a
    description of the build that is timed."""
    import tempfile

    import oracle

    if "build" not in _NATIVE:
        try:
            oracle.use_native_build(tempfile.mkdtemp(prefix="orc_native_"))
            _NATIVE["build"] = "gcc -O3 -march=native -ffp-contract=off, built on this host"
        except Exception as e:  # no compiler: the test build (-O2) is timed instead
            _NATIVE["build"] = "gcc -O2 -ffp-contract=off (native build failed: %s)" % e
    return _NATIVE["build"]


def _cpu_time(fn, budget):
    """Seconds per call of fn over about `budget` seconds (at least one call)."""
    fn()
    reps, t0 = 0, time.time()
    while True:
        fn()
        reps += 1
        if time.time() - t0 >= budget:
            break
    return (time.time() - t0) / reps, reps


def _relerr(np, x, ref):
    d = x - ref
    return float(max(np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max()))


def _cfg3(H, torch, np, synth, args):
    """Heterogeneous 100^3 diffusion (sigma 2), ILUT(1e-3, 10): FP64 factors
    against FP32 factors with FP64 refinement, FGMRES(30) to 1e-10."""
    import oracle

    A = synth.diffusion3d(100, None, None, 2.0, seed=3)
    n = A.n
    Aop = H.hec_from_csr(A)
    b = torch.from_numpy(synth.rhs(n, 1, 3)).cuda()
    res, xs = {}, {}
    for fdt in ("f64", "f32"):
        _log("config 3: ILUT setup, %s factors" % fdt)
        t0 = time.time()
        f = H.ilu_setup(A, "ilut", p=10, tol=1e-3, factor_dtype=fdt, tune=_tune(H, args))
        setup = time.time() - t0
        pl, pu = H.ilu_plans(f)
        stl, stu = H.tri_plan_stats(pl), H.tri_plan_stats(pu)
        sv = 8 if fdt == "f64" else 4
        B = counted_bytes(n, stl["nnz_offdiag"], stu["nnz_offdiag"], 1, sv=sv)
        z = torch.empty_like(b)
        _log("config 3: timing applies (%s)" % fdt)
        ms = _time_apply(H, torch, f, b, z, args.steps, args.warmup)
        row = {"apply_ms": round(ms, 4), "apply_GBps": round(B / (ms * 1e-3) / 1e9, 3),
               "counted_bytes_per_apply": int(B), "roofline": _roofline(stl, B, ms),
               "nlev_L": stl["nlev"], "nlev_U": stu["nlev"], "nnz_offdiag_L": stl["nnz_offdiag"],
               "nnz_offdiag_U": stu["nnz_offdiag"], "ell_width_L": stl["ell_width"],
               "nnz_tail_L": stl["nnz_tail"], "setup_s": round(setup, 3)}
        if not args.no_krylov:
            _log("config 3: FGMRES (%s)" % fdt)
            xs[fdt], row["fgmres"] = _krylov(H, torch, f, Aop, b, "fgmres")
        if fdt == "f64" and not args.no_cpu_baseline:
            # the oracle's substitution on the same factors (the host factors
            # are the oracle's, bit for bit)
            L = synth.CSR(n, *H.ilu_factor(f, 0))
            U = synth.CSR(n, *H.ilu_factor(f, 1))
            rr = b.cpu().numpy()
            build = _native_oracle()
            cs, reps = _cpu_time(lambda: oracle.ilu_apply(L, U, rr), args.cpu_seconds / 5)
            row["parity_relerr_vs_oracle"] = _relerr(np, z.cpu().numpy(), oracle.ilu_apply(L, U, rr))
            res["cpu_baseline"] = {"value": round(B / cs / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                                   "sample": "%d full L+U applications of the 100^3 ILUT system (serial C "
                                             "substitution, FP64 factors)" % reps,
                                   "seconds_per_apply": round(cs, 5), "build": build}
        res[fdt] = row
    out = {"workload": "heterogeneous 3D 7-point diffusion 100^3 (n=1000000), lognormal sigma=2 seed 3, "
                       "ILUT(tol 1e-3, p 10), 1 RHS; FGMRES(30) to 1e-10",
           "fp64": res["f64"], "fp32_refined": res["f32"], "cpu_baseline": res.get("cpu_baseline")}
    if not args.no_krylov:
        out["fp32_time_ratio_vs_fp64"] = round(res["f32"]["fgmres"]["seconds"] / res["f64"]["fgmres"]["seconds"], 4)
        out["rel_diff_fp32_vs_fp64_solution"] = (xs["f32"] - xs["f64"]).norm().item() / xs["f64"].norm().item()
    return out


def _cfg4(H, torch, np, synth, args):
    """RAS on the 128^3 Poisson matrix: 64 seeded contiguous subdomains,
    overlap 1, ILU(0) per subdomain in FP32, 16 RHS; FP64 BiCGSTAB."""
    import oracle

    A = synth.poisson3d(128)
    n = A.n
    owner, _ = synth.subdomain_cuts(n, 64, 8192, 61440, seed=4)
    R = 16
    _log("config 4: RAS setup")
    t0 = time.time()
    s = H.ras_setup(A, 64, owner, overlap=1, factor_dtype="f32", tune=_tune(H, args, max_nrhs=R))
    setup = time.time() - t0
    nsub, tot, ext = H.ras_info(s)
    pl, pu = H.ras_plans(s)
    stl, stu = H.tri_plan_stats(pl), H.tri_plan_stats(pu)
    # FP32 factor side on the extended rows, FP64 gather of r and prolongation of z
    B = (stl["nnz_offdiag"] + stu["nnz_offdiag"]) * 8 + tot * 4 + 2 * 4 * tot + R * (2 * tot * 4 + 2 * n * 8)
    r = torch.from_numpy(synth.rhs(n, R, 4)).cuda()
    z = torch.empty_like(r)
    _log("config 4: timing applies")
    reps = max(5, args.steps // 2)
    ms = _time_apply(H, torch, s, r, z, reps, 2, ras=True)
    out = {"workload": "RAS on 128^3 Poisson (n=2097152): 64 seeded contiguous subdomains (8192..61440 rows), "
                       "overlap 1, ILU(0) per subdomain in FP32, 16 RHS; FP64 BiCGSTAB to 1e-10",
           "apply_ms": round(ms, 4), "apply_GBps": round(B / (ms * 1e-3) / 1e9, 3), "counted_bytes_per_apply": int(B),
           "solves_per_s": round(1000.0 * R / ms, 2), "roofline": _roofline(dict(stl, nrhs=R), B, ms),
           "extended_rows": int(tot), "nlev_L": stl["nlev"], "nlev_U": stu["nlev"], "setup_s": round(setup, 3),
           "parts_L": stl["num_groups"]}
    zg = torch.empty_like(r)
    out["apply_ms_graph_replay"] = round(_graph_ms(H, torch, s, r, zg, reps), 4)
    torch.cuda.synchronize()
    out["graph_equals_eager"] = bool(torch.equal(zg, z))
    if not args.no_krylov:
        _log("config 4: BiCGSTAB")
        _, out["bicgstab"] = _krylov(H, torch, s, H.hec_from_csr(A), r, "bicgstab")
    if not args.no_cpu_baseline:
        _log("config 4: CPU oracle")
        build = _native_oracle()
        doms32 = oracle.ras_to_f32(oracle.ras_setup(A, owner, 64, overlap=1))
        rr = r.cpu().numpy()
        ref = oracle.ras_apply_f32(doms32, rr)
        out["parity_relerr_vs_oracle"] = _relerr(np, z.cpu().numpy(), ref)
        t0 = time.time()
        oracle.ras_apply_f32(doms32, rr)
        cs = time.time() - t0
        out["cpu_baseline"] = {"value": round(B / cs / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                               "sample": "1 full RAS application, 64 subdomains x 16 RHS (serial C substitution "
                                         "per subdomain, FP32)", "seconds_per_apply": round(cs, 4), "build": build}
    return out


def _cfg5(H, torch, np, synth, args):
    """256 independent systems (log-uniform 1e3..2e5 rows, 2D/3D lognormal
    sigma 1), ILU(1), 8 RHS each: FP64 factors against FP32 factors with FP64
    refinement; batched FGMRES(30), every (system, rhs) its own problem."""
    import oracle

    _log("config 5: generating systems")
    shapes = synth.batch_systems(256, seed=5)
    mats = []
    for i, (dim, side) in enumerate(shapes):
        if dim == 2:
            mats.append(synth.diffusion2d(side, None, 1.0, seed=5000 + i))
        else:
            mats.append(synth.diffusion3d(side, None, None, 1.0, seed=5000 + i))
    A, sys_ptr = _block_diag(mats)
    n = A.n
    R = 8
    b = torch.from_numpy(synth.rhs(n, R, 5)).cuda()
    Aop = H.hec_from_csr(A)
    res = {}
    z32 = None
    tuned = None
    for fdt in ("f64", "f32"):
        _log("config 5: batch ILU(1) setup, %s factors" % fdt)
        t0 = time.time()
        tune = _tune(H, args, max_nrhs=R) if tuned is None else tuned
        f = H.batch_setup(A, sys_ptr, "iluk", k=1, factor_dtype=fdt, tune=tune)
        setup = time.time() - t0
        pl, pu = H.ilu_plans(f)
        stl, stu = H.tri_plan_stats(pl), H.tri_plan_stats(pu)
        sv = 8 if fdt == "f64" else 4
        B = counted_bytes(n, stl["nnz_offdiag"], stu["nnz_offdiag"], R, sv=sv)
        z = torch.empty_like(b)
        _log("config 5: timing applies (%s)" % fdt)
        reps = max(5, args.steps // 2)
        ms = _time_apply(H, torch, f, b, z, reps, 2)
        row = {"apply_ms": round(ms, 4), "apply_GBps": round(B / (ms * 1e-3) / 1e9, 3),
               "counted_bytes_per_apply": int(B), "roofline": _roofline(dict(stl, nrhs=R), B, ms),
               "solves_per_s": round(1000.0 * len(mats) * R / ms, 1),
               "nlev_L": stl["nlev"], "nlev_U": stu["nlev"], "setup_s": round(setup, 3), "parts_L": stl["num_groups"]}
        zg = torch.empty_like(b)
        row["apply_ms_graph_replay"] = round(_graph_ms(H, torch, f, b, zg, reps), 4)
        torch.cuda.synchronize()
        row["graph_equals_eager"] = bool(torch.equal(zg, z))
        if not args.no_krylov:
            _log("config 5: batched FGMRES, one problem per (system, rhs) (%s)" % fdt)
            _, kr = _krylov_batch(H, torch, f, Aop, sys_ptr, b, "fgmres")
            row["fgmres"] = kr
            row["systems_per_s"] = round(len(mats) * R / kr["seconds"], 3)
        if fdt == "f32" and tuned is not None:
            row["autotune"] = tune_info
        res[fdt] = row
        if fdt == "f32":
            z32 = z.cpu().numpy()
        if fdt == "f64" and not args.no_autotune:
            # the FP32 plans take the tuner's choice for this batch (kernel,
            # wavefronts, parts, ELL width), searched on L's pattern within a
            # time budget; results are cached by a signature of the problem
            import tempfile

            _log("config 5: autotuning the FP32 triangular plans")
            Lf = synth.CSR(n, *H.ilu_factor(f, 0))
            t0 = time.time()
            tuned, us = H.tri_autotune(Lf, "lower", unit_diag=True, dtype="f32", nrhs=R, sys_ptr=sys_ptr,
                                       cache=os.path.join(tempfile.gettempdir(), "hec_tune_cache.jsonl"),
                                       max_seconds=40.0)
            tune_info = {"seconds": round(time.time() - t0, 2), "best_L_solve_us": round(us, 1),
                         "schedule": int(tuned.schedule), "kernel_variant": int(tuned.kernel_variant),
                         "block_threads": int(tuned.block_threads), "ell_width": int(tuned.ell_width),
                         "part_rows": int(tuned.part_rows), "partition": int(tuned.partition)}
    out = {"workload": "256 independent systems (log-uniform 1e3..2e5 rows, 2D/3D lognormal sigma=1, n=%d), ILU(1), "
                       "8 RHS each; batched FGMRES(30), each (system, rhs) to 1e-10" % n,
           "systems": len(mats), "fp64": res["f64"], "fp32_refined": res["f32"]}
    if not args.no_krylov:
        out["fp32_speedup_vs_fp64_time_to_1e-10"] = round(res["f64"]["fgmres"]["seconds"] /
                                                         res["f32"]["fgmres"]["seconds"], 4)
    if not args.no_cpu_baseline:
        _log("config 5: CPU oracle on a sample of systems")
        build = _native_oracle()
        pick = list(range(0, len(mats), 16))
        rr = b.cpu().numpy()
        bs, ts, errs = 0, 0.0, []
        for s_ in pick:
            M = mats[s_]
            L, U = oracle.iluk(M, 1)
            L32, U32 = oracle.to_f32(L), oracle.to_f32(U)
            seg = slice(int(sys_ptr[s_]), int(sys_ptr[s_ + 1]))
            t0 = time.time()
            ref = oracle.ilu_apply_f32(L32, U32, rr[seg])
            ts += time.time() - t0
            bs += counted_bytes(M.n, L.nnz - M.n, U.nnz - M.n, R, sv=4)
            errs.append(_relerr(np, z32[seg], ref))
        out["parity_relerr_vs_oracle_sampled"] = max(errs)
        out["cpu_baseline"] = {"value": round(bs / ts / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                               "sample": "%d of the 256 systems (every 16th), one FP32 L+U application with 8 RHS "
                                         "each (serial C substitution)" % len(pick),
                               "seconds": round(ts, 4), "build": build}
    return out


def run_config(cfg, args):
    """Secondary workloads (one JSON line each): 3 = mixed precision on
    heterogeneous ILUT, 4 = RAS with 16 RHS, 5 = 256 batched systems,
    6 = the block-preconditioner table of the paper's Example 1, 7 = SOR /
    Gauss-Seidel smoother sweeps."""
    import numpy as np
    import torch

    import paper_1606_00541_amd as H
    import synth

    torch.cuda.set_device(0)
    out = {"metric": "L+U solve GB/s & solves/s, FP64 vs FP32+refine/batched, at 1e-10 rel resid",
           "unit": "GB/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "config": {}}
    if cfg in (3, 4, 5):
        d = {3: _cfg3, 4: _cfg4, 5: _cfg5}[cfg](H, torch, np, synth, args)
        main = d if cfg == 4 else d["fp32_refined"]
        out.update({"value": main["apply_GBps"], "ms_per_step": main["apply_ms"],
                    "dtype": "f32 factors, f64 refinement" if cfg != 4 else "f32 factors, f64 outer",
                    "config": {"workload": d["workload"]}, "roofline": main["roofline"],
                    "cpu_baseline": d.get("cpu_baseline"), "detail": d})
    elif cfg == 6:
        out.update(_table1(H, torch, np, synth, args))
    elif cfg == 7:
        out.update(_smoother(H, torch, np, synth, args))
    else:
        raise SystemExit("unknown --config %d" % cfg)
    print(json.dumps(out))
    return 0


def _smoother(H, torch, np, synth, args):
    """SOR / Gauss-Seidel sweeps on the 128^3 Poisson matrix: a forward
    sweep is one SpMV with U + (1 - 1/omega) D and one level-scheduled lower
    solve with D/omega + L; a symmetric sweep adds the mirrored pair."""
    s = args.grid
    A = synth.poisson3d(s)
    n = A.n
    res = {}
    b = torch.from_numpy(synth.rhs(n, 1, 7)).cuda()
    for omega in (1.0, 1.5):
        _log("config 7: SOR setup, omega %.1f" % omega)
        t0 = time.time()
        S = H.sor_setup(A, omega, tune=_tune(H, args))
        setup = time.time() - t0
        nnz_off = (A.nnz - n) // 2
        nnz_n = nnz_off + (0 if omega == 1.0 else n)
        # SpMV: values + indices, read x and b, write t; solve: as one triangular launch
        B_fwd = nnz_n * 12 + 3 * n * 8 + per_launch_bytes(n, nnz_off, 1, diag=True)
        row = {"setup_s": round(setup, 3)}
        for sym in (False, True):
            x = torch.zeros_like(b)
            for _ in range(args.warmup):
                H.sor_apply(S, b, x, sweeps=1, symmetric=sym)
            torch.cuda.synchronize()
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            H.sor_apply(S, b, x, sweeps=args.steps, symmetric=sym)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            Bs = B_fwd * (2 if sym else 1)
            row["ssor" if sym else "sor"] = {"ms_per_sweep": round(ms, 4), "GBps": round(Bs / (ms * 1e-3) / 1e9, 2)}
        if not args.no_cpu_baseline:
            import oracle

            x0 = synth.rhs(n, 1, 8)
            xt = torch.from_numpy(x0.copy()).cuda()
            H.sor_apply(S, b, xt, sweeps=1, symmetric=True)
            t2 = time.time()
            ref = oracle.sor(A, b.cpu().numpy(), x0, omega=omega, sweeps=1, symmetric=True)
            row["cpu_oracle_ms_per_ssor_sweep"] = round(1e3 * (time.time() - t2), 3)
            row["parity_relerr_vs_oracle"] = float(np.linalg.norm(xt.cpu().numpy() - ref) / np.linalg.norm(ref))
        res["omega_%.1f" % omega] = row
    gs = res["omega_1.0"]["sor"]
    return {"value": gs["GBps"], "dtype": "f64", "ms_per_step": gs["ms_per_sweep"],
            "config": {"workload": "SOR / Gauss-Seidel smoother on 3D 7-point Poisson %d^3 (n=%d), FP64, 1 RHS; "
                                   "step = one forward Gauss-Seidel sweep (SpMV + level-scheduled lower solve)"
                                   % (s, n)},
            "sweeps": res}


# Block counts and one-application times ("Pre GPU (s)") of the paper's
# Example 1 table (3D Poisson, n = 1,000,000; Tesla C2050, FP64): context
# from another machine, not a target.
_TABLE1_PAPER = {("BILU", 16): 0.0057, ("BILU", 128): 0.0055, ("BILU", 512): 0.0052,
                 ("BILUT", 16): 0.010, ("BILUT", 128): 0.011, ("BILUT", 512): 0.010,
                 ("RAS", 256): 0.0051, ("RAS", 2048): 0.0056}


def _table1(H, torch, np, synth, args):
    """The shape of the paper's Example 1 table: 3D Poisson 100^3, GMRES(20)
    to 1e-10 in FP64 with block ILU(0) and block ILUT(7, 0.1) on 16/128/512
    geometric blocks, and RAS (overlap 1, ILU(0)) on 256/2048 subdomains.  Per
    row: one preconditioner application on the GPU (HIP events), the serial
    CPU oracle's application on a small sample, and the whole GPU solve."""
    import oracle

    s = 100
    A = synth.poisson3d(s)
    n = A.n
    Aop = H.hec_from_csr(A)
    b = torch.from_numpy(synth.rhs(n, 1, 6)).cuda()
    rows = []
    for pre, nb in (("BILU", 16), ("BILU", 128), ("BILU", 512), ("BILUT", 16), ("BILUT", 128), ("BILUT", 512),
                    ("RAS", 256), ("RAS", 2048)):
        owner = synth.grid_bisection(s, s, s, nb)
        kind, kw, ov = ("ilut", {"p": 7, "tol": 0.1}, 0) if pre == "BILUT" else ("ilu0", {}, 1 if pre == "RAS" else 0)
        _log("config 6: %s %d setup" % (pre, nb))
        t0 = time.time()
        M = H.ras_setup_ilu(A, nb, owner, overlap=ov, kind=kind, tune=_tune(H, args), **kw)
        setup = time.time() - t0
        nsub, tot, _ = H.ras_info(M)
        pl, pu = H.ras_plans(M)
        stl, stu = H.tri_plan_stats(pl), H.tri_plan_stats(pu)
        # FP64 factors on the extended rows, FP64 gather of r and prolongation of z
        B = (stl["nnz_offdiag"] + stu["nnz_offdiag"]) * 12 + tot * 8 + 2 * 4 * tot + (2 * tot * 8 + 2 * n * 8)
        z = torch.empty_like(b)
        ms = _time_apply(H, torch, M, b, z, args.steps, args.warmup, ras=True)
        _log("config 6: %s %d GMRES(20)" % (pre, nb))
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t1 = time.time()
        st, info = H.krylov_solve(Aop, M, b, x, method="gmres", m=20, rtol=1e-10)
        torch.cuda.synchronize()
        solve = time.time() - t1
        row = {"pre": pre, "blocks": nb, "setup_s": round(setup, 3), "extended_rows": int(tot),
               "nlev_L": stl["nlev"], "nlev_U": stu["nlev"], "dataflow": stl["dataflow"],
               "pre_gpu_ms": round(ms, 4), "pre_GBps": round(B / (ms * 1e-3) / 1e9, 2),
               "gmres20": {"status": int(st), "iters": info[0].iters, "relres": info[0].relres,
                           "seconds": round(solve, 4)},
               "paper_pre_gpu_ms_c2050": 1e3 * _TABLE1_PAPER[(pre, nb)]}
        if not args.no_cpu_baseline:
            _log("config 6: %s %d CPU oracle application" % (pre, nb))
            okw = {"p": 7, "tau": 0.1} if kind == "ilut" else {}
            doms = oracle.ras_setup(A, owner, nb, overlap=ov, kind=kind, **okw)
            rr = synth.rhs(n, 1, 6)
            t2 = time.time()
            zr = oracle.ras_apply(doms, rr)
            row["pre_cpu_oracle_ms"] = round(1e3 * (time.time() - t2), 3)
            row["parity_relerr_vs_oracle"] = float(np.linalg.norm(z.cpu().numpy() - zr) / np.linalg.norm(zr))
        rows.append(row)
    first = rows[0]
    return {"value": first["pre_GBps"], "dtype": "f64", "ms_per_step": first["pre_gpu_ms"],
            "config": {"workload": "3D 7-point Poisson 100^3 (n=1000000, nnz 6,940,000), GMRES(20) to 1e-10, "
                                   "FP64; BILU/BILUT(7, 0.1) on 16/128/512 and RAS(overlap 1) on 256/2048 "
                                   "geometric-bisection blocks; value = BILU-16 application GB/s"},
            "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--schedule", default="auto",
                    choices=["auto", "level_launch", "level_persistent", "owner_persistent"])
    ap.add_argument("--kernel-variant", type=int, default=0,
                    help="hec_tune_t.kernel_variant (0 = auto: the dataflow kernel when it fits)")
    ap.add_argument("--block-threads", type=int, default=0, help="hec_tune_t.block_threads (0 = default)")
    ap.add_argument("--no-krylov", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="config 5: default tuning instead of the autotuner")
    ap.add_argument("--timed-loop-only", action="store_true",
                    help="skip the device refactorization and the per-application (warm/cold) timings, so a "
                         "profiler sees only the warmup and timed applications")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="default run: skip the sub-results of configs 3, 4 and 5")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (for counter calibration)")
    ap.add_argument("--config", type=int, default=2,
                    help="2 (default): 128^3 ILU(0) L+U; 3: mixed precision ILUT; 4: RAS 16 RHS; 5: batch")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print("bench.py measures one GPU: the level-scheduled solve of one system does not shard "
              "across GPUs (every level would need an exchange); run with --gpus 1", file=sys.stderr)
        return 2

    if args.config != 2:
        return run_config(args.config, args)

    import numpy as np
    import torch

    import paper_1606_00541_amd as H
    import synth

    torch.cuda.set_device(0)
    s = args.grid
    A = synth.poisson3d(s)
    n = A.n
    t0 = time.time()
    f = H.ilu_setup(A, "ilu0", tune=_tune(H, args))
    setup_s = time.time() - t0
    pl, pu = H.ilu_plans(f)
    stl, stu = H.tri_plan_stats(pl), H.tri_plan_stats(pu)
    r = torch.from_numpy(synth.rhs(n, 1, 2)).cuda()
    z = torch.empty_like(r)
    stream = torch.cuda.current_stream()

    B = counted_bytes(n, stl["nnz_offdiag"], stu["nnz_offdiag"], 1)
    for _ in range(args.warmup):
        H.ilu_apply(f, r, z)
    torch.cuda.synchronize()
    # HIP events on the stream the kernels are launched on (torch's current stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        H.ilu_apply(f, r, z)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gbs = B / (ms * 1e-3) / 1e9
    # numeric refactorization on the device with the same values: the first
    # call builds the pattern maps, later calls reuse them
    refac = refac_first = refac_same = reps = reps_cold = None
    if not args.timed_loop_only:
        refac, refac_first, refac_same, reps, reps_cold = _extras(H, torch, np, f, A, r, z, stream, args)

    # dominant kernel: the triangular-solve kernel; L and U launches share it
    bl = per_launch_bytes(n, stl["nnz_offdiag"], 1, diag=False)
    bu = per_launch_bytes(n, stu["nnz_offdiag"], 1, diag=True)
    if stl["syncfree"] and stu["syncfree"]:
        kname, tag = "k_syncfree", "syncfree"
        launches = 2
    elif stl["schedule"] == 1:
        kname, tag = "k_level", "launch"
        launches = stl["nlev"] + stu["nlev"]
    elif stl["dataflow"] and stu["dataflow"]:
        kname, tag = "k_dataflow", "dataflow"
        launches = 2
    elif stl["schedule"] == 3 and stl["nnz_tail"] == 0 and stu["nnz_tail"] == 0:
        kname, tag = "k_owner", "owner"
        launches = 2
    else:
        kname, tag = "k_persistent", "level" if stl["schedule"] == 2 else "owner"
        launches = 2
    per_launch = (bl + bu) / launches
    kernel_ms = ms / launches
    achieved = per_launch / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(kname, "poisson%d_ilu0_f64_%s" % (s, tag))
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "algorithmic_bytes_per_launch": int(per_launch),
                "traffic": None if traffic is None else int(traffic)}

    out = {
        "metric": "L+U solve GB/s & solves/s, FP64 vs FP32+refine/batched, at 1e-10 rel resid",
        "value": round(gbs, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D 7-point Poisson %d^3 (n=%d), ILU(0) FP64, HEC ELL width %d, 1 RHS U[-1,1] "
                               "seed 2; step = one L+U preconditioner application" % (s, n, stl["ell_width"]),
                   "n": n, "nnz_offdiag_L": stl["nnz_offdiag"], "nnz_offdiag_U": stu["nnz_offdiag"],
                   "nlev_L": stl["nlev"], "nlev_U": stu["nlev"], "schedule": args.schedule,
                   "kernel": kname, "crit_hops_L": stl["crit_hops"],
                   "workgroups": stl["num_groups"], "counted_bytes_per_step": int(B),
                   "setup_s": round(setup_s, 3),
                   "device_refactor_ms": None if refac is None else round(1e3 * refac, 3),
                   "device_refactor_first_call_s": None if refac_first is None else round(refac_first, 3),
                   "refactor_bit_identical": refac_same},
        "solves_per_s": round(1000.0 / ms, 2),
        "per_rep_ms": {"warm": reps, "cold": reps_cold},
        "roofline": roofline,
    }

    if args.calibrate_copy_mib > 0:
        src = torch.empty(args.calibrate_copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = int(src.numel() * 8)

    if not args.no_krylov:
        M = H.hec_from_csr(A)
        b = torch.from_numpy(synth.rhs(n, 1, 2)).cuda()
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t1 = time.time()
        st, info = H.krylov_solve(M, f, b, x, method="gmres", m=30, rtol=1e-10)
        torch.cuda.synchronize()
        ks = time.time() - t1
        out["krylov"] = {"method": "GMRES(30)+ILU(0)", "status": int(st), "iters": info[0].iters,
                         "precond_applies": info[0].precond_applies, "relres": info[0].relres,
                         "seconds": round(ks, 4), "systems_per_s": round(1.0 / ks, 4)}
        # the same solve with FP32 factors and FP64 refinement (flexible GMRES)
        f32 = H.ilu_setup(A, "ilu0", factor_dtype="f32", tune=_tune(H, args))
        z32 = torch.empty_like(r)
        ms32 = _time_apply(H, torch, f32, r, z32, args.steps, args.warmup)
        x32 = torch.zeros_like(b)
        torch.cuda.synchronize()
        t1 = time.time()
        st32, info32 = H.krylov_solve(M, f32, b, x32, method="fgmres", m=30, rtol=1e-10)
        torch.cuda.synchronize()
        ks32 = time.time() - t1
        out["krylov_fp32_refined"] = {
            "method": "FGMRES(30)+ILU(0), FP32 factors, FP64 outer", "status": int(st32),
            "iters": info32[0].iters, "relres": info32[0].relres, "seconds": round(ks32, 4),
            "apply_ms": round(ms32, 5), "time_ratio_vs_fp64": round(ks32 / ks, 4),
            "rel_diff_vs_fp64_solution": (x32 - x).norm().item() / x.norm().item()}

    if not args.no_cpu_baseline:
        import oracle

        L, U = oracle.ilu0(A)
        rr = synth.rhs(n, 1, 2)
        z_test_build = oracle.ilu_apply(L, U, rr)
        build = _native_oracle()
        oracle.ilu_apply(L, U, rr)  # warm
        reps, t2 = 0, time.time()
        while time.time() - t2 < args.cpu_seconds:
            oracle.ilu_apply(L, U, rr)
            reps += 1
        cs = (time.time() - t2) / reps
        zr = oracle.ilu_apply(L, U, rr)
        err = float(np.linalg.norm(z.cpu().numpy() - zr) / np.linalg.norm(zr))
        out["cpu_baseline"] = {"value": round(B / cs / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                               "sample": "%d full L+U applications of the same %d^3 system (serial C "
                                         "substitution on CSR, natural order)" % (reps, s),
                               "seconds_per_apply": round(cs, 5), "build": build,
                               "identical_to_test_build": bool(np.array_equal(zr, z_test_build))}
        out["parity_relerr_vs_oracle"] = err
        # multithreaded level-scheduled CPU solve (Algorithm 2 on all host
        # cores), bit-identical to the serial substitution above
        sl, su = oracle.LevelSolveCPU(L, unit=True), oracle.LevelSolveCPU(U, upper=True)
        zp = su.solve(sl.solve(rr))
        reps, t2 = 0, time.time()
        while time.time() - t2 < args.cpu_seconds / 3:
            su.solve(sl.solve(rr))
            reps += 1
        cp = (time.time() - t2) / reps
        out["cpu_levels_omp"] = {"value": round(B / cp / 1e9, 4), "unit": "GB/s", "cores": oracle.omp_threads(),
                                 "kind": "level-scheduled OpenMP CPU solve",
                                 "sample": "%d full L+U applications of the same system" % reps,
                                 "seconds_per_apply": round(cp, 5),
                                 "bit_identical_to_oracle": bool(np.array_equal(zp, zr))}
    if not args.no_secondary:
        # the metric's FP32+refinement and batched halves, on the other
        # workloads of the benchmark family (each with its own roofline and
        # CPU oracle baseline)
        out["secondary"] = {"config3_ilut_mixed_precision": _cfg3(H, torch, np, synth, args),
                            "config4_ras_16rhs": _cfg4(H, torch, np, synth, args),
                            "config5_batch256": _cfg5(H, torch, np, synth, args)}
    out["paper_context"] = ("paper (Tesla C2050 vs Xeon X5570, FP64): triangular solves ~7x, "
                            "linear solver ~10x; another machine, not a target")
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
