"""Build liblbpf.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1902_08933_amd.build   (or call build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbpf.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]

SOURCES = ["lbpf_kernels.hip", "lbpf_api.cpp", "lbpf_unet_kernels.hip", "lbpf_unet.cpp", "lbpf_sp.hip",
           "lbpf_d3q15.hip"]
# Per-source device flags. The MFMA kernels keep their accumulators in VGPRs (the VGPR form of
# the MFMA instructions): otherwise the compiler holds loop-carried accumulators in VGPRs and
# copies them to AGPRs and back around every MFMA block.
SOURCE_FLAGS = {"lbpf_unet_kernels.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, jobs=None):
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + COMMON + DEVICE_FLAGS + SOURCE_FLAGS.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    bad = [src for p, src in procs if p.wait() != 0]
    if bad:
        raise RuntimeError("hipcc failed for " + ", ".join(bad))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC"] + DEVICE_FLAGS + ["-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
