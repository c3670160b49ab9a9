"""The library's host code under AddressSanitizer (CPU, no GPU needed).

Builds every source of libmh with the sanitizer on the host pass only (the
device code is compiled as usual and never runs here), links it with
tests/asan_host_driver.cpp and runs the driver: workspace arithmetic for
single samples, two node sets and batches, and every argument and workspace
check that precedes the first kernel, with the caller's host arrays in heap
blocks of exactly their stated length.  Any out-of-bounds access or use after
free in that host code fails the test."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2509_13230_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
ROCM_LIB = "/opt/rocm/lib"
# the sanitizer applies to the host pass only (the flag pair must stay together)
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(CLANG) or shutil.which(B.hipcc()) is None and not os.path.exists(B.hipcc()):
        pytest.skip("ROCm clang / hipcc not available")
    out = tmp_path_factory.mktemp("asan")

    def compile_one(src):
        obj = str(out / (os.path.splitext(src)[0] + ".o"))
        cmd = [B.hipcc(), *B.HIPCC_FLAGS, *HOST_ASAN, "-I", B.INCLUDE, "-I", B.CSRC, "-c",
               os.path.join(B.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        return obj, r

    with ThreadPoolExecutor(min(6, os.cpu_count() or 1)) as ex:
        built = list(ex.map(compile_one, B.SOURCES))
    for obj, r in built:
        assert r.returncode == 0, r.stderr[-2000:]
    drv_o = str(out / "driver.o")
    r = subprocess.run([CLANG, "-O1", "-fsanitize=address", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
                        "-I", B.INCLUDE, "-I", "/opt/rocm/include", "-c", os.path.join(HERE, "asan_host_driver.cpp"),
                        "-o", drv_o], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(out / "asan_host_driver")
    r = subprocess.run([CLANG, "-fsanitize=address", drv_o, *[o for o, _ in built], "-L", ROCM_LIB, "-lamdhip64",
                        "-Wl,-rpath," + ROCM_LIB, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def test_host_code_under_asan(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([driver], capture_output=True, text=True, timeout=120, env=env)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "0 failed" in r.stdout
