"""Build the HIP solver library (gfx950) in-tree: paper_2604_23951_amd/_lib/liblpgpu.so, and
its checked build (bounds checks in the product kernels, LPGPU_CHECKED=1) liblpgpu_checked.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "liblpgpu.so")
CHECKED_LIB_PATH = os.path.join(LIB_DIR, "liblpgpu_checked.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("lp_kernels.hip", "lp_api.cpp", "lp_layout.cpp", "lp_presolve.cpp")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # every multiply and add rounded on its own, so the elementwise updates match their
    # plain definition bit for bit
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def build(verbose: bool = False, checked: bool = False) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    path = CHECKED_LIB_PATH if checked else LIB_PATH
    tmp = path + ".tmp"
    # (the checks' atomics keep a few unrolled loops of the panel kernel rolled: expected)
    extra = ["-DLPGPU_CHECKED=1", "-Wno-pass-failed"] if checked else []
    cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{out}")
    if verbose and out.strip():
        print(out, file=sys.stderr)
    os.replace(tmp, path)
    return path


if __name__ == "__main__":
    print(build(verbose=True))
    print(build(verbose=True, checked=True))
