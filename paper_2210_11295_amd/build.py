"""Build the gfx950 HIP library libbsrht.so in-tree (paper_2210_11295_amd/_lib).

Every csrc/*.hip file is compiled with hipcc for gfx950 and linked into one
shared library exporting the C ABI of include/bsrht.h.  Packed FP32 vector
instructions are disabled for all device code.
"""

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB_NAME = "libbsrht.so"
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON_FLAGS = [
    "-O3", "-std=c++20", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]

# Per-file device code generation options.  The dense kernels keep MFMA
# accumulators in ordinary VGPRs: with AGPR accumulators the FP64 GEMM copies
# all of them between the two register files on every k tile and needs more
# than 256 registers, which leaves one wave per SIMD.
FILE_FLAGS = {
    "dense.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
}


def _compile(src, obj_dir):
    obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON_FLAGS + FILE_FLAGS.get(os.path.basename(src), []) + [
        "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build_library(jobs=8, verbose=False):
    """Compile all sources and link libbsrht.so; returns the library path."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    os.makedirs(OUT_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(lambda s: _compile(s, obj_dir), srcs))
    out = os.path.join(OUT_DIR, LIB_NAME)
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build_library(verbose=True)
