"""Host code under the address and undefined-behaviour sanitizers (CPU only).

* The oracle (oracle/oracle.c, FP64 and FP32) built with gcc
  -fsanitize=address,undefined runs every entry point on small grids
  (heat with every boundary, the adjoints, Euler with every scheme variant and
  wall, the CFL step, the plane sums): tests/sanitize/oracle_driver.c.
* The C ABI's argument validation (capi.cpp, and hetero.cpp which it links)
  built with the same host sanitizers (hipcc, -Xarch_host before each
  sanitizer flag, so the device side is built without them), linked with
  stand-ins for the kernel launchers, runs every entry point's error paths
  and the valid workspace-size queries: tests/sanitize/capi_driver.cpp.

Either run must end with status 0 and no sanitizer report."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(cmd, cwd):
    p = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout}\n{p.stderr}"
    return p


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    flags = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
             "-fopenmp", "-std=c11", "-ffp-contract=off"]
    objs = []
    for real, sfx in (("double", "_f64"), ("float", "_f32")):
        obj = str(tmp_path / f"oracle{sfx}.o")
        _run(["gcc"] + flags + [f"-DREAL={real}", f"-DSFX={sfx}", "-c", os.path.join(ROOT, "oracle", "oracle.c"),
                                "-o", obj], tmp_path)
        objs.append(obj)
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc"] + flags + [os.path.join(SAN, "oracle_driver.c")] + objs + ["-lm", "-o", exe], tmp_path)
    p = _run([exe], tmp_path)
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr


def test_capi_validation_under_host_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain not found")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-sanitize-recover=all"]
    base = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include")]
    objs = []
    for src in (os.path.join(ROOT, "paper_2105_10332_amd", "csrc", "capi.cpp"),
                os.path.join(ROOT, "paper_2105_10332_amd", "csrc", "hetero.cpp"),
                os.path.join(SAN, "capi_stubs.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run(base + san + ["-x", "hip", "-c", src, "-o", obj], tmp_path)
        objs.append(obj)
    drv = str(tmp_path / "drv.o")
    hostsan = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    _run([CLANG, "-O1", "-g", "-std=c++17"] + hostsan + ["-I", os.path.join(ROOT, "include"), "-c",
                                                           os.path.join(SAN, "capi_driver.cpp"), "-o", drv], tmp_path)
    exe = str(tmp_path / "capi_driver")
    _run([CLANG] + hostsan + [drv] + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
         tmp_path)
    p = _run([exe], tmp_path)
    assert "0 failures" in p.stdout
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr
