"""CPU-only checks of the C ABI: the library loads, exports every function that
include/abac.h declares, and its host-side validation works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abac.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abac_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_03574_amd.abac import load_library, LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2306_03574_amd.build import build
        build()
    return load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("abac_plan_create", "abac_apply_A", "abac_apply_Pinv", "abac_minres_solve"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2306_03574_amd.abac import EXPORTED
    names = _declared()
    assert sorted(EXPORTED) == names
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("nx,ny,nt,ok", [
    (63, 0, 64, True), (255, 255, 256, True), (4095, 0, 1024, True), (127, 63, 128, True),
    (64, 0, 64, False), (63, 0, 60, False), (63, 0, 4, False), (1023, 1023, 64, False),
    (8191, 0, 64, False), (63, 62, 64, False), (63, 0, 2048, False),
])
def test_workspace_bytes_validation(lib, nx, ny, nt, ok):
    n = lib.abac_workspace_bytes(nx, ny, nt, 0, 1)
    assert (n > 0) == ok
    if ok:
        N = nt * nx * max(ny, 1)
        assert n >= 8 * 8 * N          # eight FP64 Krylov vectors at least
        assert lib.abac_workspace_bytes(nx, ny, nt, 1, 1) < n   # FP32 scratch is smaller
        assert lib.abac_workspace_bytes(nx, ny, nt, 2, 1) < lib.abac_workspace_bytes(nx, ny, nt, 1, 1)  # no scratch
        assert lib.abac_workspace_bytes(nx, ny, nt, 0, 4) > 3 * n


@pytest.mark.parametrize("args", [
    (63, 0, 64, 1.0, 0.0, 0, 1),      # alpha = 0
    (63, 0, 64, 1.0, 1.5, 0, 1),      # alpha > 1
    (63, 0, 64, -1.0, 0.1, 0, 1),     # T < 0
    (63, 0, 64, 1.0, 0.1, 3, 1),      # bad precision
    (63, 0, 64, 1.0, 0.1, 0, 0),      # batch 0
    (62, 0, 64, 1.0, 0.1, 0, 1),      # nx+1 not a power of two
])
def test_plan_create_rejects_bad_arguments_without_touching_the_gpu(lib, args):
    h = ctypes.c_void_p()
    st = lib.abac_plan_create(*args, None, None, 0, ctypes.byref(h))
    assert st == -1
    assert h.value is None
    assert len(lib.abac_last_error()) > 0


def test_status_strings(lib):
    assert lib.abac_status_string(0) == b"ok"
    assert lib.abac_status_string(-4) == b"not converged"
    assert lib.abac_status_string(-5) == b"breakdown"


@pytest.mark.parametrize("args", [
    (511, 511, 512, 1.0, 1e-3, 1, 1),   # 511^2 x 512 FP32 scratch: over the fixed array
    (255, 255, 256, 1.0, 1e-3, 0, 2),   # two FP64 right-hand sides of 255^2 x 256: over it
    (63, 0, 64, 1.0, 0.9, 0, 1),        # alpha near 1 (singularity check needs a plan)
    (63, 0, 64, 1.0, 1e-3, 2, 1),       # no transforms to apply
    (62, 0, 64, 1.0, 1e-3, 0, 1),       # nx+1 not a power of two
])
def test_noalloc_apply_rejects_without_touching_the_gpu(lib, args):
    """The allocation-free P^{-1} checks sizes and arguments on the host first; the
    pointers are never dereferenced on these paths."""
    dummy = ctypes.c_void_p(256)
    st = lib.abac_apply_Pinv_noalloc(*args, dummy, dummy, None)
    assert st == -1
    assert len(lib.abac_last_error()) > 0
