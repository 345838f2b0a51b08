"""AddressSanitizer + UndefinedBehaviorSanitizer run of the C ABI's host code.

sq_api.hip (argument checks, work list, column-major projector tables, launch
plan) is rebuilt with host-only sanitizers (device code unchanged) and linked
with the package's other objects into a temporary library; the driver
tests/sanitize_capi_driver.cpp, built with the same sanitizers, feeds it
malformed inputs (which must be refused with SQ_ERR_ARG) and valid geometries in
every boundary mode (which must build all host tables; without a GPU setup then
stops at its first device call).  A sanitizer report aborts the driver.
Skipped when the package's objects (written by build()) or the compilers are
missing."""
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2011_13517_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_capi_host_code_under_asan_ubsan(tmp_path):
    objs = [o for o in glob.glob(os.path.join(PKG, "_build", "*.o"))
            if os.path.basename(o) != "sq_api.o"]
    if not objs or not shutil.which(HIPCC) or not os.path.exists(CLANG):
        pytest.skip("package objects or compilers missing (run build() first)")
    api = str(tmp_path / "sq_api.o")
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc")] + SAN_HOST +
         ["-c", os.path.join(PKG, "csrc", "sq_api.hip"), "-o", api])
    lib = str(tmp_path / "libsq_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN_HOST[:4] +
         ["-o", lib] + sorted(objs) + [api])
    drv = str(tmp_path / "driver")
    _run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
          "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
          os.path.join(HERE, "sanitize_capi_driver.cpp"), lib, "-Wl,-rpath," + str(tmp_path),
          "-o", drv])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([drv], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
