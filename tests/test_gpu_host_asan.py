"""The host layer of the library under AddressSanitizer: a C driver of the C ABI
(tests/host_asan/abac_host_driver.cpp, built with the library's host code instrumented
by paper_2306_03574_amd.build.build_host_driver) runs plans, operators, MINRES and GMRES
solves, a variable coefficient, groups, the request server with its group lane and the
allocation-free entry point.  Any out-of-bounds access, use after free, double free or
leak of the host code ends the driver with a report and a non-zero status."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "paper_2306_03574_amd", "abac_host_driver")
SUPP = os.path.join(ROOT, "tests", "host_asan", "lsan.supp")


def test_host_layer_under_address_sanitizer():
    if not os.path.exists(DRIVER):
        pytest.skip("host driver not built (python -m paper_2306_03574_amd.build --host-driver)")
    print("[case] host driver under AddressSanitizer", flush=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={SUPP}:print_suppressions=0"
    r = subprocess.run([DRIVER], capture_output=True, text=True, timeout=240, env=env)
    tail = (r.stdout[-2000:] + "\n" + r.stderr[-6000:])
    print(tail, flush=True)
    assert "ERROR: AddressSanitizer" not in r.stderr and "ERROR: LeakSanitizer" not in r.stderr, tail
    assert r.returncode == 0, tail
    assert "HOST_DRIVER_OK" in r.stdout, tail
