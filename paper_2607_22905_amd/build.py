"""Build libalgmortar.so (gfx950) in-tree with hipcc.

    python -m paper_2607_22905_amd.build        # or build() from Python

Every source is compiled each time this runs.  HIP code is built with packed
FP32 instructions disabled.
"""
import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.environ.get("ALGMORTAR_BUILD_DIR", os.path.join(HERE, "_build"))
LIB = os.environ.get("ALGMORTAR_LIB", os.path.join(HERE, "libalgmortar.so"))

SOURCES = [
    "host_structure.cpp",
    "iface_nd.cpp",
    "algmortar_api.cpp",
    "kernels_local.hip",
    "kernels_values.hip",
    "kernels_local_f64.hip",
    "kernels_local_f32.hip",
    "kernels_local_bf16.hip",
    "kernels_iface.hip",
    "kernels_nd.hip",
    "kernels_inexact.hip",
    "kernels_pcg.hip",
    "kernels_smooth.hip",
    "kernels_tpfa.hip",
    "static_scratch.hip",
]

ARCH = os.environ.get("ALGMORTAR_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


EXTRA = os.environ.get("ALGMORTAR_CFLAGS", "").split()


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + EXTRA + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if os.environ.get("ALGMORTAR_BUILD_TIMES"):
        print(f"  {src}: {time.time() - t0:.0f} s", flush=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(9, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
