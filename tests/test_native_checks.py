"""Native checks run on the CPU:

* the kernels' square-root rounding correction, exhaustively over every float
  argument in [2^-96, FLT_MAX] (tests/native/sqrt_fix_check.cpp);
* the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer, every
  entry point on small and degenerate inputs (tests/native/oracle_sanitize.c);
* the library's host code (validation, planning, descriptor tables, workspace
  offsets, enqueueing) built for the host only with both sanitizers and run
  against a stand-in HIP runtime (tests/native/host_sanitize.cpp).
"""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2208_00001_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_sqrt_round_fix_exhaustive(tmp_path):
    exe = str(tmp_path / "sqrt_fix_check")
    _run(["g++", "-O2", "-mfma", "-fopenmp", "-ffp-contract=off", "-I", CSRC, "-o", exe,
          os.path.join(NATIVE, "sqrt_fix_check.cpp"), "-lm"])
    out = _run([exe]).stdout
    print(out)
    assert "failures 0" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-o", exe,
          os.path.join(ROOT, "oracle", "ggdt_ref.c"), os.path.join(NATIVE, "oracle_sanitize.c"), "-lm"])
    r = _run([exe], env=SAN_ENV)
    print(r.stdout)
    assert "0 failures" in r.stdout and "ERROR" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.slow
@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)), reason="needs hipcc")
def test_host_code_under_sanitizers(tmp_path):
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs.append(os.path.join(NATIVE, "host_sanitize.cpp"))
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    objs = []

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17",
              "-Wno-unused-result", *san, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
        objs = list(ex.map(compile_one, srcs))
    # the per-source device-image symbols a host-only object refers to
    nm = _run(["nm", "-u", *objs]).stdout
    fatbins = sorted({ln.split()[-1] for ln in nm.splitlines() if "__hip_fatbin_" in ln})
    stub = tmp_path / "fatbin_stubs.c"
    stub.write_text("".join(f"char {name}[1];\n" for name in fatbins))
    exe = str(tmp_path / "host_san")
    _run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, *objs, "-x", "c", str(stub)])
    r = _run([exe], env=SAN_ENV)
    print(r.stdout)
    assert "0 failures" in r.stdout and "ERROR" not in r.stderr and "runtime error" not in r.stderr
