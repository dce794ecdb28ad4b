"""The allocation-free P_alpha^{-1} entry point (abac_apply_Pinv_noalloc) against the
plan-based abac_apply_Pinv, through the C ABI, on two calls in a row on one GPU, the
second with a smaller input (the fixed device array keeps the first call's contents),
and in both transform precisions; plus its refusal of sizes beyond the array.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _pair(nx, ny, nt, alpha, prec, batch, seed):
    """(noalloc result, plan result) for a seeded input."""
    from paper_2306_03574_amd import Plan
    from paper_2306_03574_amd.abac import apply_Pinv_noalloc
    print(f"[case] noalloc nx={nx} ny={ny} nt={nt} alpha={alpha} prec={prec} batch={batch}", flush=True)
    shape = (batch, nt) + ((ny, nx) if ny else (nx,))
    r = torch.from_numpy(np.random.default_rng(seed).standard_normal(shape)).to(DEV)
    z = apply_Pinv_noalloc(r, nx, ny, nt, alpha=alpha, prec=prec)
    p = Plan(nx, ny, nt, alpha=alpha, prec=prec, batch=batch, device=DEV)
    zp = p.apply_Pinv(r)
    torch.cuda.synchronize()
    return z.cpu().numpy(), zp.cpu().numpy()


# (first call, second call with a smaller input): separate x/y passes, the fused x-y
# passes and 1D, FP64 and FP32 transforms
SEQUENCES = [
    ((255, 127, 64, 1e-3, "fp64", 1), (31, 15, 16, 1e-2, "fp64", 1)),
    ((63, 63, 128, 1e-3, "fp32", 2), (1023, 0, 16, 1e-3, "fp32", 1)),
    ((4095, 0, 256, 1e-1, "fp64", 1), (15, 15, 8, 1e-3, "fp64", 3)),
]


@pytest.mark.parametrize("first,second", SEQUENCES)
def test_noalloc_matches_plan_on_two_calls(first, second):
    for k, case in enumerate((first, second)):
        z, zp = _pair(*case, seed=100 + k)
        err = _rel(z, zp)
        print(f"[obs] noalloc vs plan rel.err {err:.3e}", flush=True)
        # FP64: same kernels, tables computed on the device instead of the host (a few
        # ulp apart); FP32: the FP32 tables round the same FP64 values
        assert err < (1e-12 if case[4] == "fp64" else 1e-5), (case, err)


def test_noalloc_refuses_more_than_its_array():
    from paper_2306_03574_amd.abac import AbacError, EINVAL, apply_Pinv_noalloc
    print("[case] noalloc oversize 511^2 x 512 fp32", flush=True)
    r = torch.zeros((1, 8, 7, 7), dtype=torch.float64, device=DEV)   # never read
    with pytest.raises(AbacError) as ei:
        # the size is checked against the declared grid before any device work
        from paper_2306_03574_amd.abac import load_library
        import ctypes
        st = load_library().abac_apply_Pinv_noalloc(511, 511, 512, 1.0, 1e-3, 1, 1, ctypes.c_void_p(r.data_ptr()),
                                                    ctypes.c_void_p(r.data_ptr()), None)
        from paper_2306_03574_amd.abac import _check
        _check(st, "abac_apply_Pinv_noalloc")
    assert ei.value.status == EINVAL and "at most" in str(ei.value)
