"""The entry point that allocates nothing (ilu_apply_noalloc): the same
results as ilu_apply, bit for bit, on two calls in a row, the second one
smaller, and a clear error past its fixed scratch."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1606_00541_amd as H  # noqa: E402
from parity import relerr  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def both(f, r):
    rt = dev(r)
    z1, z2 = torch.empty_like(rt), torch.empty_like(rt)
    H.ilu_apply(f, rt, z1)
    H.ilu_apply_noalloc(f, rt, z2)
    torch.cuda.synchronize()
    return z1.cpu().numpy(), z2.cpu().numpy()


@pytest.mark.parametrize("kernel", ["auto", "syncfree", "level_launch"])
@pytest.mark.parametrize("fdt", ["f64", "f32"])
def test_noalloc_apply_matches_ilu_apply_on_two_calls(kernel, fdt):
    kw = {}
    if kernel == "syncfree":
        kw = {"schedule": "level_launch", "kernel_variant": 5}
    elif kernel == "level_launch":
        kw = {"schedule": "level_launch"}
    A1 = synth.poisson3d(40)                       # first call: 64,000 rows, 3 RHS
    A2 = synth.diffusion2d(37, 29, 1.0, seed=7)    # second call: smaller, 1 RHS
    f1 = H.ilu_setup(A1, "ilu0", factor_dtype=fdt, tune=H.tune_default(max_nrhs=3, **kw))
    f2 = H.ilu_setup(A2, "iluk", k=1, factor_dtype=fdt, tune=H.tune_default(max_nrhs=1, **kw))
    tol = 1e-12 if fdt == "f64" else 1e-5
    r1 = synth.rhs(A1.n, 3, 11)
    z_ref, z_na = both(f1, r1)
    assert np.array_equal(z_na, z_ref)
    L, U = oracle.ilu0(A1)
    ref = oracle.ilu_apply(L, U, r1) if fdt == "f64" else oracle.ilu_apply_f32(oracle.to_f32(L), oracle.to_f32(U), r1)
    assert relerr(z_na, ref) <= tol
    r2 = synth.rhs(A2.n, 1, 12)
    z_ref, z_na = both(f2, r2)
    assert np.array_equal(z_na, z_ref)
    L, U = oracle.iluk(A2, 1)
    ref = oracle.ilu_apply(L, U, r2) if fdt == "f64" else oracle.ilu_apply_f32(oracle.to_f32(L), oracle.to_f32(U), r2)
    assert relerr(z_na, ref) <= tol


def test_noalloc_apply_rejects_what_it_cannot_hold():
    A = synth.poisson3d(128)  # 2,097,152 rows: one FP64 RHS fits, two do not
    f = H.ilu_setup(A, "ilu0", tune=H.tune_default(max_nrhs=2))
    r = dev(synth.rhs(A.n, 2, 13))
    z = torch.empty_like(r)
    with pytest.raises(H.HecError) as e:
        H.ilu_apply_noalloc(f, r, z)
    assert e.value.name == "CAPACITY"
    r1 = dev(synth.rhs(A.n, 1, 14))
    z1, z2 = torch.empty_like(r1), torch.empty_like(r1)
    H.ilu_apply_noalloc(f, r1, z1)
    H.ilu_apply(f, r1, z2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    g = H.ilu_setup(synth.poisson2d(20), "ilu0", tune=H.tune_default(max_nrhs=1))
    r3 = dev(synth.rhs(400, 2, 15))
    with pytest.raises(H.HecError) as e:  # more RHS than the handle was set up for
        H.ilu_apply_noalloc(g, r3, torch.empty_like(r3))
    assert e.value.name == "INVALID_ARG"
