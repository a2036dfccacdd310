"""The host-sanitised debugging build (build.py variant "host_asan": host
code under AddressSanitizer and UndefinedBehaviorSanitizer) runs the host
tests of the C interface cleanly.  CPU only: the ASan runtime is loaded
first through LD_PRELOAD in a child process, which a GPU run does not allow.
The device-side debugging build ("lds_nan") needs a GPU; its use is
described in build.py."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan():
    rt = asan_runtime()
    if rt is None:
        pytest.skip("no clang ASan runtime in this image")
    from paper_1704_08897_amd import build as B
    lib = B.variant_path("host_asan")
    src = max(os.path.getmtime(os.path.join(B.CSRC, s)) for s in B.SOURCES)
    if not os.path.exists(lib) or os.path.getmtime(lib) < src:
        B.build(variant="host_asan")
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in nm and "__ubsan_handle" in nm      # really instrumented
    env = dict(os.environ, LD_PRELOAD=rt, BHX_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_capi_host.py", "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-3000:]
