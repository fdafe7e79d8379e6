"""AddressSanitizer and UndefinedBehaviorSanitizer runs of the host code, on
the CPU.

* The FP64 oracle (plain C): every entry point over small grids of every
  lattice, with walls, moving walls, obstacles, a force field, a mass source,
  both forcing schemes and the 16-bit storage emulation, and its refused
  arguments (tests/native/oracle_sanitize.c).
* The host side of the library's C ABI (mdf_api.cpp: case validation,
  workspace layout and size limits, the refused forms of mdf_init, NULL
  contexts), compiled under the sanitizers and linked with the kernels'
  objects as built (tests/native/host_sanitize.cpp).  No call reaches the
  device.

Either run stops at the first out-of-bounds access, use after free, leak,
signed overflow or invalid conversion, and the test fails with its report.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2108_08591_amd", "csrc")
ROCM = "/opt/rocm"
SAN = ["-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed:\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    _run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Wno-unknown-pragmas", *SAN, "-I", os.path.join(ROOT, "oracle"),
          "-o", exe, os.path.join(NATIVE, "oracle_sanitize.c"), "-lm"])
    r = _run([exe], env=_env(), timeout=300)
    assert "32 cases, 0 failed checks" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(f"{ROCM}/lib/libamdhip64.so"),
                    reason="g++ or the HIP runtime not available")
def test_host_library_under_sanitizers(tmp_path):
    objs = sorted(o for o in glob.glob(os.path.join(CSRC, "_build", "*.o")) if "mdf_api" not in os.path.basename(o))
    if len(objs) < 3:
        pytest.skip("kernel objects not built (paper_2108_08591_amd/build.py)")
    api = str(tmp_path / "mdf_api.o")
    drv = str(tmp_path / "host_sanitize.o")
    exe = str(tmp_path / "host_sanitize")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", f"{ROCM}/include", *inc, "-c",
          os.path.join(CSRC, "mdf_api.cpp"), "-o", api])
    _run(["g++", "-std=c++17", *SAN, *inc, "-c", os.path.join(NATIVE, "host_sanitize.cpp"), "-o", drv])
    _run(["g++", *SAN, "-o", exe, drv, api, *objs, f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"])
    r = _run([exe], env=_env(), timeout=300)
    assert "0 failed checks" in r.stdout
