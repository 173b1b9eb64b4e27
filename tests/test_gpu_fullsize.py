"""GPU parity at the benchmark shapes, element by element against the oracle.

Each workload is built exactly as bench.py builds it and solved in the launch
configuration bench.py times (the automatic choice), plus the forced kernel
that configuration can fall back to.  The oracle finishes each of these in
seconds, so every output element is compared (tests/parity.py: normwise and
element-wise relative error).

Tolerances: FP64 factors 1e-12 (level order, the folded reciprocal diagonal
and fused multiply-adds change only the rounding); FP32 factors solved in
FP32 1e-5 against the oracle's FP32 substitution (a few units of the FP32
rounding, 6e-8, times the growth along a few hundred levels).
"""
import numpy as np
import pytest

import oracle
import synth
from synth import CSR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1606_00541_amd as H  # noqa: E402
from parity import relerr  # noqa: E402

F64_TOL, F32_TOL = 1e-12, 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def apply(f, r, ras=False):
    rt = dev(r)
    zt = torch.empty_like(rt)
    (H.ras_apply if ras else H.ilu_apply)(f, rt, zt)
    torch.cuda.synchronize()
    return zt.cpu().numpy()


def block_diag(mats):
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


@pytest.mark.parametrize("variant", [0, 4])
def test_config2_poisson128_fp32_factors(variant):
    # 128^3 Poisson, ILU(0) rounded once to FP32, FP64 vectors
    A = synth.poisson3d(128)
    f = H.ilu_setup(A, "ilu0", factor_dtype="f32",
                    tune=H.tune_default(kernel_variant=variant,
                                        schedule="owner_persistent" if variant else "auto"))
    assert H.tri_plan_stats(H.ilu_plans(f)[0])["dataflow"] == 1
    L, U = oracle.ilu0(A)
    r = synth.rhs(A.n, 1, 2)
    z = apply(f, r)
    assert relerr(z, oracle.ilu_apply_f32(oracle.to_f32(L), oracle.to_f32(U), r)) <= F32_TOL


@pytest.fixture(scope="module")
def config3():
    A = synth.diffusion3d(100, None, None, 2.0, seed=3)
    L, U = oracle.ilut(A, 10, 1e-3)
    return A, L, U


@pytest.mark.parametrize("fdt", ["f64", "f32"])
def test_config3_ilut_sigma2_full_size(config3, fdt):
    # 100^3 lognormal (sigma 2) diffusion, ILUT(tol 1e-3, p 10): factors bit
    # for bit, then the application on the dataflow kernel (ELL width covering
    # the longest row)
    A, L, U = config3
    f = H.ilu_setup(A, "ilut", p=10, tol=1e-3, factor_dtype=fdt)
    for w, T in ((0, L), (1, U)):
        rp, ci, v = H.ilu_factor(f, w)
        assert np.array_equal(rp, T.rowptr) and np.array_equal(ci, T.col) and np.array_equal(v, T.val)
    pl, pu = H.ilu_plans(f)
    sl, su = H.tri_plan_stats(pl), H.tri_plan_stats(pu)
    assert sl["dataflow"] == 1 and su["dataflow"] == 1
    assert sl["ell_width"] in (10, 12, 16) and sl["nnz_tail"] == 0
    r = synth.rhs(A.n, 1, 3)
    z = apply(f, r)
    if fdt == "f64":
        assert relerr(z, oracle.ilu_apply(L, U, r)) <= F64_TOL
    else:
        assert relerr(z, oracle.ilu_apply_f32(oracle.to_f32(L), oracle.to_f32(U), r)) <= F32_TOL


@pytest.fixture(scope="module")
def config4():
    A = synth.poisson3d(128)
    owner, _ = synth.subdomain_cuts(A.n, 64, 8192, 61440, seed=4)
    doms = oracle.ras_setup(A, owner, 64, overlap=1)
    r = synth.rhs(A.n, 16, 4)
    ref = oracle.ras_apply_f32(oracle.ras_to_f32(doms), r)
    return A, owner, doms, r, ref


@pytest.mark.parametrize("kernel", ["auto", "syncfree", "level_launch"])
def test_config4_ras64_16rhs_fp32_full_size(config4, kernel):
    A, owner, doms, r, ref = config4
    kw = {"syncfree": {"schedule": "level_launch", "kernel_variant": 5},
          "level_launch": {"schedule": "level_launch"}}.get(kernel, {})
    s = H.ras_setup(A, 64, owner, overlap=1, factor_dtype="f32", tune=H.tune_default(max_nrhs=16, **kw))
    assert list(H.ras_info(s)[2]) == [len(d.ext) for d in doms]
    z = apply(s, r, ras=True)
    assert relerr(z, ref) <= F32_TOL


@pytest.fixture(scope="module")
def config5():
    shapes = synth.batch_systems(256, seed=5)
    mats = []
    for i, (dim, side) in enumerate(shapes):
        if dim == 2:
            mats.append(synth.diffusion2d(side, None, 1.0, seed=5000 + i))
        else:
            mats.append(synth.diffusion3d(side, None, None, 1.0, seed=5000 + i))
    A, sys_ptr = block_diag(mats)
    L, U = oracle.iluk(A, 1)  # block diagonal: the ILU(1) of every system at once
    r = synth.rhs(A.n, 8, 5)
    ref = oracle.ilu_apply_f32(oracle.to_f32(L), oracle.to_f32(U), r)
    return A, sys_ptr, r, ref


@pytest.mark.parametrize("kernel", ["auto", "syncfree"])
def test_config5_batch256_iluk1_8rhs_fp32_full_size(config5, kernel):
    A, sys_ptr, r, ref = config5
    kw = {"schedule": "level_launch", "kernel_variant": 5} if kernel == "syncfree" else {}
    f = H.batch_setup(A, sys_ptr, "iluk", k=1, factor_dtype="f32", tune=H.tune_default(max_nrhs=8, **kw))
    z = apply(f, r)
    assert relerr(z, ref) <= F32_TOL
    # and per system (each scaled by its own size)
    for s in range(len(sys_ptr) - 1):
        seg = slice(int(sys_ptr[s]), int(sys_ptr[s + 1]))
        assert relerr(z[seg], ref[seg]) <= F32_TOL
