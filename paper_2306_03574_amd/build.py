"""Build the HIP library ``libabac.so`` for gfx950 in-tree (next to this file).

Usage: ``python -m paper_2306_03574_amd.build`` (or ``build()`` from Python);
``--host-driver`` also builds the C-ABI driver whose host code runs under
AddressSanitizer (``build_host_driver()``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libabac.so")
SOURCES = ["abac_api.hip", "kernels_stencil.hip", "kernels_transform.hip", "kernels_small.hip", "kernels_gmres.hip",
           "kernels_gen.hip", "server.hip", "group.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed FP32 vector ops are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fuse within one source expression only (the language rule), never
    # across statements: a device function then rounds the same way in every kernel it
    # is inlined into, so solves advanced in a group match their solo runs bitwise
    "-ffp-contract=on",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, csrc: str = CSRC, lib: str = LIB) -> str:
    """Compile every source into libabac.so (always recompiles).  The translation
    units compile in parallel to objects in a temporary folder, then link."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    cc = hipcc()
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="abac_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[cc] + flags + ["-c", os.path.join(csrc, s), "-o", o] for s, o in zip(SOURCES, objs)]
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for c, res in zip(cmds, results):
            if verbose:
                print(" ".join(c), flush=True)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed compiling {c[-3]}")
        tmp = lib + ".tmp"
        link = [cc, "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libabac.so")
        os.replace(tmp, lib)
    return lib


HOST_DRIVER = os.path.join(HERE, "abac_host_driver")
HOST_DRIVER_SRC = os.path.join(os.path.dirname(HERE), "tests", "host_asan", "abac_host_driver.cpp")
# AddressSanitizer for the host code only (device code stays uninstrumented)
HOST_ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_driver(verbose: bool = False, csrc: str = CSRC, out: str = HOST_DRIVER) -> str:
    """Compile the C-ABI driver of tests/host_asan together with every library source
    into one executable whose host code runs under AddressSanitizer (always rebuilds).
    The translation units compile in parallel, then link."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    cc = hipcc()
    flags = [f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC")] + HOST_ASAN_FLAGS
    srcs = [os.path.join(csrc, s) for s in SOURCES] + [HOST_DRIVER_SRC]
    with tempfile.TemporaryDirectory(prefix="abac_asan_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(os.path.basename(s))[0] + ".o") for s in srcs]
        cmds = [[cc] + flags + ["-c", s, "-o", o] for s, o in zip(srcs, objs)]
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for c, res in zip(cmds, results):
            if verbose:
                print(" ".join(c), flush=True)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed compiling {c[-3]}")
        link = [cc, "--offload-arch=gfx950"] + HOST_ASAN_FLAGS + objs + ["-o", out + ".tmp"]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking the host driver")
        os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    if "--host-driver" in sys.argv:
        print(build_host_driver(verbose=True))
