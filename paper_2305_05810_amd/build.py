"""Build libstf.so (HIP, gfx950) in-tree.

Every source is compiled with -ffp-contract=off (the tap choice is pinned
binary32 arithmetic; fused multiply-adds are written out where wanted) and
with packed-FP32 instructions disabled.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
TARGET = os.path.join(HERE, "libstf.so")
ARCH = os.environ.get("STF_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-bitwise-instead-of-logical", "-I", os.path.join(HERE, "..", "include")]

# Per-file additions.  The neural-texture inference kernel reads its MFMA
# results with ordinary VALU instructions, so the results go to architectural
# VGPRs instead of accumulation registers (saves a copy per value).  Its 168
# VGPRs (3 waves per SIMD) hold the MLP as operand images; the scheduler's
# register-pressure trackers keep it within them (0 bytes of scratch instead
# of 12-16 spilled bytes per lane, and 3% faster).
EXTRA = {"neural.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form", "-mllvm", "-amdgpu-use-amdgpu-trackers=1"]}


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), sources()))
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", TARGET + ".tmp", *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(TARGET + ".tmp", TARGET)
    return TARGET


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
