"""Build libwvprime.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("wv_kernels.hip", "wv_capi.hip", "wv_tune.hip", "wv_server.hip",
                                                 "wv_irregular.hip", "wv_static.hip")]
PEAK_SRC = os.path.join(HERE, "csrc", "peak.hip")
PEAK_LIB = os.path.join(HERE, "libwvpeak.so")
DEPS = [os.path.join(HERE, "csrc", f) for f in ("mont.hpp", "sum_core.hpp", "wv_tables.hpp", "wv_internal.hpp",
                                                "wv_ctx.hpp")] + [
    os.path.join(ROOT, "include", "wvprime.h")]
LIB = os.path.join(HERE, "libwvprime.so")
ARCH = os.environ.get("WV_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off in every HIP build of this package
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # fully unrolled difference-table loops keep a stale unroll request
    "-Wno-pass-failed",
]


def _hipcc(srcs, out, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + f".tmp{os.getpid()}"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose=False):
    """Compile the HIP sources in SRCS into libwvprime.so and the
    instruction-rate microbenchmarks csrc/peak.hip into libwvpeak.so (both
    gfx950, in-tree)."""
    _hipcc(SRCS, LIB, verbose)
    _hipcc([PEAK_SRC], PEAK_LIB, verbose)
    return LIB


def is_stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in [*SRCS, *DEPS])


if __name__ == "__main__":
    print(build(verbose=True))
