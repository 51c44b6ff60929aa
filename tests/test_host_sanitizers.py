"""The library's host code (planner, argument validation, plane-wave helper)
built with AddressSanitizer and UndefinedBehaviorSanitizer on the host side
only, and driven by tests/host_check.cpp without a device.  The device code
is the regular build's (linked from its objects)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2501_13512_amd")
OBJ = os.path.join(ROOT, "_build")
SAN = os.path.join(OBJ, "sanitize")
DEVICE_OBJS = ["mvm.o", "krylov.o", "block_solver.o", "fields.o", "gmres.o"]
# -fsanitize reaches the host compilation only (each one after -Xarch_host)
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_host_code_under_asan_and_ubsan():
    if not all(os.path.exists(os.path.join(OBJ, o)) for o in DEVICE_OBJS):
        from paper_2501_13512_amd import build
        build.build()
    os.makedirs(SAN, exist_ok=True)
    from paper_2501_13512_amd.build import FLAGS
    api_obj = os.path.join(SAN, "vie_api_san.o")
    _run([_hipcc(), *FLAGS, *SAN_FLAGS, "-x", "hip", "-c", os.path.join(PKG, "csrc", "vie_api.cpp"), "-o", api_obj])
    drv_obj = os.path.join(SAN, "host_check.o")
    _run([_hipcc(), "-O1", "-std=c++17", "-I" + os.path.join(ROOT, "include"), *SAN_FLAGS, "-x", "c++", "-c",
          os.path.join(ROOT, "tests", "host_check.cpp"), "-o", drv_obj])
    exe = os.path.join(SAN, "host_check")
    _run([_hipcc(), "--offload-arch=gfx950", *SAN_FLAGS, drv_obj, api_obj,
          *[os.path.join(OBJ, o) for o in DEVICE_OBJS], "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "host_check ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
