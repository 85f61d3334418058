"""Host code under sanitizers, and the workspace lease (CPU, no GPU).

- The oracle's C code, built with AddressSanitizer and UndefinedBehavior-
  Sanitizer, runs every entry point on exact-size buffers around the word
  boundaries (tests/oracle_asan_driver.c).
- libpa's host code (planner, tuning table and its file parser, argument
  validation, serving scheduler with the simulated executor, driven from
  several threads) is built with AddressSanitizer on its host pass and run
  by tests/libpa_asan_driver.c.  Nothing here launches a kernel.
- The stream workspace lease (csrc/pa_workspace.h) on a simulated stream:
  several host threads share one stream while the buffer grows; no work
  item may find its buffer freed (tests/workspace_lease_test.cpp).  The
  same program releasing the lease before enqueueing (the unsafe order)
  must be caught, which shows the check can fail.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_07592_amd", "csrc")
TESTS = os.path.join(ROOT, "tests")
ROCM_CLANG = "/opt/rocm/llvm/bin/clang"


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-6000:])
    return r


def test_workspace_lease_on_a_simulated_stream(tmp_path):
    exe = str(tmp_path / "wlt")
    run(["g++", "-std=c++17", "-O1", "-pthread", "-I", CSRC, os.path.join(TESTS, "workspace_lease_test.cpp"),
         "-o", exe])
    out = run([exe], timeout=120).stdout
    assert '"after_free": 0' in out and '"failures": 0' in out
    # releasing the lease before the work is enqueued is detected
    run([exe, "early"], timeout=120)


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    run(["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "toeplitz_oracle.c"),
         os.path.join(TESTS, "oracle_asan_driver.c"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="4")
    out = run([exe], env=env, timeout=300).stdout
    assert '"failures": 0' in out


LIB_SOURCES = ["pa_kernels.hip", "pa_plan.cpp", "pa_api.cpp", "pa_serve.cpp", "pa_tune.cpp", "pa_graph.cpp",
               "pa_fft.hip", "pa_fft_host.cpp", "pa_probe.hip", "pa_noalloc.hip"]


@pytest.mark.skipif(not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")) or
                    not os.path.exists(ROCM_CLANG), reason="needs the ROCm toolchain")
def test_libpa_host_code_under_asan(tmp_path):
    from paper_1809_07592_amd import build as B
    hipcc = B.hipcc()
    # the sanitizer flags apply to the host pass only (the device code is
    # compiled as usual, so the library loads, but nothing here runs it)
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        run([hipcc] + flags + ["-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, LIB_SOURCES))
    lib = str(tmp_path / "libpa_asan.so")
    run([hipcc, "--offload-arch=gfx950", "-shared", "-Xarch_host", "-fsanitize=address", "-o", lib] + objs)
    exe = str(tmp_path / "libpa_asan_driver")
    run([ROCM_CLANG, "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-pthread",
         "-I", os.path.join(ROOT, "include"), os.path.join(TESTS, "libpa_asan_driver.c"), lib,
         "-Wl,-rpath," + str(tmp_path), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               LD_LIBRARY_PATH=str(tmp_path) + ":/opt/rocm/lib:" + os.environ.get("LD_LIBRARY_PATH", ""),
               HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    env.pop("PA_TUNE_CACHE", None)
    env.pop("PA_HBM_BUDGET", None)
    out = run([exe, str(tmp_path)], env=env, timeout=300).stdout
    assert '"failures": 0' in out
