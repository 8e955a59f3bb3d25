"""The allocation-free blob mobility product (arb_rpy_apply_noalloc_dev) against
the allocating one (arb_rpy_apply_dev), through the C ABI, on two calls in a
row, the second smaller (the scratch keeps the first call's contents).

With the target-parallel kernel and the same source slices both entry points
run the same kernels in the same order: bit for bit equal.  With the
autotuned allocating product (possibly the symmetric kernel) the bar is the
product's own: 1e-12 relative L2 in FP64, 1e-5 in FP32C (Sec. 2.3 Eq. RPY).
"""
import numpy as np
import pytest

from paper_2107_10800_amd import arb
from paper_2107_10800_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def run(ctx, pos, lam, fn):
    import torch

    N = pos.shape[0]
    pd = torch.tensor(pos.ravel(), dtype=torch.float64, device="cuda")
    ld = torch.tensor(lam.ravel(), dtype=torch.float64, device="cuda")
    ud = torch.full((3 * N,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    fn(ctx, N, pd, ld, ud)
    torch.cuda.synchronize()
    return ud.cpu().numpy()


@pytest.mark.parametrize("prec", [arb.ARB_FP64, arb.ARB_FP32C])
@pytest.mark.parametrize("wall", [True, False])
def test_noalloc_matches_allocating_product(prec, wall):
    bar = 1e-12 if prec == arb.ARB_FP64 else 1e-5
    same = arb.arb_create(precision=prec, wall=wall, pair_kernel=arb.ARB_PAIR_TARGET, slices=4)
    auto = arb.arb_create(precision=prec, wall=wall)
    try:
        for N, seed, box in ((9000, 3, 80.0), (1234, 4, 30.0)):
            cl = W.random_blobs(N, seed=seed, box=box)
            pos, lam = cl["pos"], cl["lam"]
            print(f"noalloc prec={prec} wall={wall} N={N}", flush=True)
            u_na = run(same, pos, lam, arb.arb_rpy_apply_noalloc_dev)
            u_ref = run(same, pos, lam, arb.arb_rpy_apply_dev)
            assert np.all(np.isfinite(u_na))
            assert np.array_equal(u_na, u_ref)
            u_na2 = run(auto, pos, lam, arb.arb_rpy_apply_noalloc_dev)
            u_auto = run(auto, pos, lam, arb.arb_rpy_apply_dev)
            e = rel(u_na2, u_auto)
            print(f"  vs autotuned product: {e:.2e}", flush=True)
            assert e <= bar
    finally:
        arb.arb_destroy(same)
        arb.arb_destroy(auto)


def test_noalloc_limits():
    import torch

    ctx = arb.arb_create(precision=arb.ARB_FP64, wall=True)
    fmm = arb.arb_create(precision=arb.ARB_FP64, pair_kernel=arb.ARB_PAIR_FMM)
    try:
        buf = torch.zeros(3, dtype=torch.float64, device="cuda")
        assert arb.arb_rpy_apply_noalloc_dev(ctx, 0, buf, buf, buf) == arb.ARB_OK
        with pytest.raises(arb.ArbError) as e:
            arb.arb_rpy_apply_noalloc_dev(ctx, arb.ARB_NOALLOC_MAX_BLOBS + 1, buf, buf, buf)
        assert e.value.code == arb.ARB_E_ARG and "maximum" in str(e.value)
        with pytest.raises(arb.ArbError) as e:
            arb.arb_rpy_apply_noalloc_dev(fmm, 1, buf, buf, buf)
        assert e.value.code == arb.ARB_E_ARG
    finally:
        arb.arb_destroy(ctx)
        arb.arb_destroy(fmm)
