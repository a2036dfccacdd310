"""Build the HIP library ``libbhx.so`` in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbhx.so")
SOURCES = ["bhx_kernels.hip", "bhx_direct.hip", "bhx_noalloc.hip", "bhx_runtime.cpp",
           "bhx_capi.cpp", "bhx_engine.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # kernel arguments arrive preloaded in SGPRs (gfx950): the batch pointer
    # is there at wave start, one round trip less before the first load
    "-mllvm", "-amdgpu-kernarg-preload-count=8",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed: {' '.join(cmd[-3:])}")
    if verbose and r.stderr.strip():
        # the host pass does not know the packed-fp32 feature; that warning is harmless
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            print("\n".join(lines))


# Debugging builds, each a library of its own beside libbhx.so (load one with
# BHX_LIB=<path> in the environment of the process that imports the binding):
#   lds_nan     every transform kernel fills its dynamic LDS with NaN before
#               use, so reads of LDS no thread wrote poison the results;
#   host_asan   host code (runtime, engine, C interface) under AddressSanitizer
#               and UndefinedBehaviorSanitizer; device code unchanged.  The
#               ASan runtime must be loaded first (LD_PRELOAD of the clang
#               runtime), so this one is for host-only test runs on a CPU
#               machine (tests/test_debug_builds.py).
VARIANTS = {
    "lds_nan": ["-DBHX_DEBUG_LDS_NAN=1"],
    "host_asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan"],
}


def variant_path(variant):
    return os.path.join(HERE, f"libbhx_{variant}.so")


def build(verbose=False, extra=(), variant=None):
    """Compile every source to an object (in parallel), then link
    ``libbhx.so`` (or ``libbhx_<variant>.so`` for a debugging variant);
    raises on failure."""
    from concurrent.futures import ThreadPoolExecutor
    inc = ["-I", os.path.join(HERE, "..", "include")]
    objdir = os.path.join(HERE, "_build", variant or "release")
    if variant:
        extra = list(extra) + VARIANTS[variant]
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        jobs.append((obj, [HIPCC, *compile_flags, *extra, *inc, "-c",
                           os.path.join(CSRC, src), "-o", obj]))
    workers = min(len(jobs), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda j: _run(j[1], verbose), jobs))
    out = variant_path(variant) if variant else LIB
    tmp = out + ".tmp"
    _run([HIPCC, *FLAGS, *extra, *[o for o, _ in jobs], "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, variant=sys.argv[1] if len(sys.argv) > 1 else None))
