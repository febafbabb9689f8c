"""Host sanitizers on the C ABI: every library source is built with
AddressSanitizer and UndefinedBehaviorSanitizer on its host side (the device
code is compiled as usual and never run), linked with
tests/abi_sanitize_driver.c, and the driver's descriptor validation, group-map
parsing, workspace layouts and rejections must run clean.  No GPU is used:
every call the driver makes returns before the library's first HIP call."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2011_04736_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

# Host-side instrumentation only: each sanitizer flag goes to the host pass.
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not available")
def test_abi_host_code_clean_under_asan_ubsan(tmp_path):
    from paper_2011_04736_amd import _build
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([HIPCC, *flags, *HOST_SAN, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(_build.SOURCES))) as ex:
        objs = list(ex.map(compile_one, _build.SOURCES))
    drv = str(tmp_path / "driver.o")
    r = subprocess.run([CLANG, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", f"-I{os.path.join(ROOT, 'include')}", "-c",
                        os.path.join(HERE, "abi_sanitize_driver.c"), "-o", drv], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "abi_asan")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *HOST_SAN[:4], drv, *objs, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # The HIP runtime keeps process-lifetime allocations: leak reports are off.
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout
