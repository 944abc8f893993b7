"""Build libhsim.so (HIP for gfx950) in-tree with hipcc.

Flags: -O3; -ffp-contract=off (the double-precision validation mode relies on
separately rounded operations; the single-precision path writes its fused
multiply-adds explicitly); packed FP32 instructions disabled for device code.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libhsim.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["sweep_kernels.hip", "rep_kernels.hip", "energy_kernels.hip", "analysis_kernels.hip",
           "output_kernels.hip", "plan.cpp", "batch.cpp", "api.cpp"]
ARCH = os.environ.get("HSIM_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall",
          "-Wno-unused-result", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]


def _compile(src, build_dir=BUILD, defines=()):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    cmd = ["hipcc"] + COMMON + list(defines) + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False, out=OUT, build_dir=BUILD, defines=()):
    """Compile every source and link libhsim.so; returns its path.  defines:
    extra -D flags (e.g. tile shape), out/build_dir: where to put the result."""
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        results = list(ex.map(lambda src: _compile(src, build_dir, defines), SOURCES))
    if verbose:
        for _, err in results:
            if err.strip():
                sys.stderr.write(err)
    objs = [o for o, _ in results]
    tmp = out + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
