"""Build libgett.so (HIP for gfx950) in-tree.

    python -m paper_2410_06770_amd.build

Every source compiles with hipcc for gfx950 only; packed-FP32 instructions are
disabled for all device code (they are known to misbehave on this part).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.environ.get("GETT_LIB_OUT") or os.path.join(HERE, "libgett.so")
# The checked build: every gathered and every C element is tested against its
# tensor's addressed range (GETT_ADDR_CHECK); for tests, not for speed.
CHECK_OBJ = os.path.join(HERE, "_build_check")
CHECK_LIB = os.path.join(HERE, "libgett_check.so")

SOURCES = ["gett_tile_f64.hip", "gett_tile_f32.hip", "gett_tile_bf3.hip", "gett_bf3pack.hip",
           "gett_ozaki.hip",
           "gett_tile_z64.hip",
           "gett_tile_c32.hip", "gett_fp8.hip",
           "gett_mlp.hip", "gett_noalloc.hip", "gett_scale.hip", "gett_unary.hip",
           "gett_unary.cpp", "gett_dispatch.cpp", "gett_plan.cpp", "gett_host.cpp"]
# Per-file code generation: the FP64, FP32, complex, packed, Ozaki and FP8
# kernels keep their MFMA accumulators in ordinary VGPRs (no per-step copies to the
# accumulation registers, lower register totals and higher occupancy); the
# direct BF16x3 tiles do better with the default form.
FILE_FLAGS = {
    "gett_tile_f64.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "gett_tile_f32.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "gett_tile_z64.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "gett_tile_c32.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "gett_bf3pack.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "gett_ozaki.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "gett_fp8.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


EXTRA = os.environ.get("GETT_EXTRA_FLAGS", "").split()


def _compile(src: str, objdir: str, defs: list) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(objdir, src + ".o")
    if src.endswith(".hip"):
        cmd = ["hipcc", "-x", "hip", *DEVICE, *COMMON, *defs, *FILE_FLAGS.get(src, []), *EXTRA,
               "-c", path, "-o", obj]
    else:
        cmd = ["hipcc", *COMMON, *defs, "-c", path, "-o", obj]
    subprocess.check_call(cmd)
    return obj


def _build(objdir: str, lib: str, defs: list, verbose: bool) -> str:
    os.makedirs(objdir, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, objdir, defs), SOURCES))
    tmp = lib + ".tmp"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


def build(verbose: bool = False, check: bool = True) -> str:
    """Build libgett.so, and the checked libgett_check.so unless check=False."""
    _build(OBJ, LIB, [], verbose)
    if check:
        _build(CHECK_OBJ, CHECK_LIB, ["-DGETT_ADDR_CHECK"], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
