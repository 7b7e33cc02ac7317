"""Host code under the compilers' sanitizers, on the CPU.

  * the oracle's C part built with gcc -fsanitize=address,undefined, loaded
    into a Python that preloads the sanitizer runtimes, running the oracle's
    pin tests;
  * libzm's host code (every translation unit, device code built as usual)
    built with address + undefined-behaviour sanitizers on the host side
    only, and again with the thread sanitizer, linked into
    tests/host_abi_check.c, which exercises the host functions, the argument
    checks of every entry point and the thread-local error text from 8
    threads.

No GPU is involved: the entry points are called only with arguments they
must reject before any device call.  The serving scheduler is pure Python
on one thread (its native calls are the entry points above), so the thread
sanitizer run covers the native state it relies on: the plan and batch
bookkeeping behind a mutex, the tune cache and the thread-local errors.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2304_14492_amd", "csrc")
SOURCES = ["plan.cpp", "zrp_table.hip", "polar_fft.hip", "project.hip", "reconstruct.hip", "batch.hip",
           "cartesian.hip", "resample.hip", "diag.cpp"]
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.slow


def _gcc_runtime(name):
    return subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()


def test_oracle_pins_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    so = str(tmp_path / "_zm_oracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-shared", "-fPIC", "-o", so, os.path.join(ROOT, "oracle", "zm_oracle.c"), "-lm"])
    env = dict(os.environ)
    env.update(LD_PRELOAD=_gcc_runtime("libasan.so") + ":" + _gcc_runtime("libubsan.so"),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               ZM_ORACLE_SO=so, OMP_NUM_THREADS="4")
    check = f"import oracle; assert oracle._SO == {so!r}; oracle._lib()"
    subprocess.check_call([sys.executable, "-c", check], cwd=ROOT, env=env)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_oracle_zrp.py",
                        "tests/test_oracle_moments.py", "tests/test_oracle_reconstruct.py",
                        "tests/test_oracle_golden.py", "tests/test_dedup.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]


def _build_libzm_host(tmp_path, san_flags):
    objs = []

    def one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
        for f in san_flags + ["-fno-omit-frame-pointer"]:
            cmd += ["-Xarch_host", f]
        cmd += ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        subprocess.run(cmd, check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(one, SOURCES))
    harness = str(tmp_path / "harness.o")
    subprocess.check_call([CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
                           "-c", os.path.join(ROOT, "tests", "host_abi_check.c"), "-o", harness] + san_flags)
    exe = str(tmp_path / "host_abi_check")
    subprocess.check_call([CLANGXX, harness] + objs + ["-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-lpthread",
                                                       "-Wl,-rpath,/opt/rocm/lib"] + san_flags)
    return exe


@pytest.mark.parametrize("san", [["-fsanitize=address", "-fsanitize=undefined"], ["-fsanitize=thread"]],
                         ids=["asan_ubsan", "tsan"])
def test_libzm_host_code_under_sanitizers(tmp_path, san):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("ROCm compilers missing")
    exe = _build_libzm_host(tmp_path, san)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 failure(s)" in out
    assert "WARNING: ThreadSanitizer" not in out and "runtime error" not in out, out[-4000:]
