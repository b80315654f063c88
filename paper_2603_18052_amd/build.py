"""Build liblindblad.so (HIP, gfx950) in-tree: one hipcc -c per source in
parallel, then one link; also the standalone device probes in probes/bin.
Usage: python -m paper_2603_18052_amd.build"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC_DIR = os.path.join(HERE, "csrc")
OBJ_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblindblad.so")
PROBE_DIR = os.path.join(HERE, "probes")  # standalone device probes (executables in probes/bin)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


# Per-source flags.  The per-step INT8 GEMM keeps 120 int32 accumulators live
# across its k loop; with the default accumulator-register form the compiler
# renames them through AGPR moves every chunk (126 v_accvgpr moves per 84
# MFMAs), with the VGPR form the MFMAs accumulate in place (d = 27, B = 1024:
# 47.1 -> 43.8 us per step).  The same form measured faster for the FP64
# build products (64 d = 27 builds 53.3 -> 47.5 ms) and the FP64 / FP32
# per-step GEMMs (ring FP64 82.8 -> 80.3 us, B = 64 16.4 -> 15.3 us); the
# BF16 fused chain's files keep the default (hi+lo measured 2 % slower).
VGPR_FORM = ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
EXTRA_FLAGS = {
    "chain_i8_large.hip": VGPR_FORM,
    "chain_large.hip": VGPR_FORM,
    "zgemm.hip": VGPR_FORM,
}


def _compile(src: str) -> str:
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    deps = [src, os.path.abspath(__file__)] + glob.glob(os.path.join(SRC_DIR, "*.hpp")) + \
        [os.path.join(HERE, "..", "include", "lindblad.h")]
    if os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps):
        return obj
    cmd = [HIPCC, *FLAGS, *EXTRA_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _probe(src: str) -> str:
    exe = os.path.join(PROBE_DIR, "bin", os.path.splitext(os.path.basename(src))[0])
    if os.path.exists(exe) and os.path.getmtime(exe) >= os.path.getmtime(src):
        return exe
    r = subprocess.run([HIPCC, *FLAGS, src, "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return exe


def build(force: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    os.makedirs(os.path.join(PROBE_DIR, "bin"), exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(SRC_DIR, "*.hip")))
    probes = sorted(glob.glob(os.path.join(PROBE_DIR, "*.hip")))
    if force:
        for o in glob.glob(os.path.join(OBJ_DIR, "*.o")) + glob.glob(os.path.join(PROBE_DIR, "bin", "*")):
            os.remove(o)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
        list(ex.map(_probe, probes))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
