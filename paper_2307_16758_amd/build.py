"""Build libswe.so for gfx950 in-tree: g++ for the host mesh toolkit,
hipcc for the device runtime.  ``python paper_2307_16758_amd/build.py``
(run as a script: importing the package itself needs the built library)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswe.so")
ARCH = os.environ.get("SWE_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             # no packed FP32 instructions anywhere in the device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # FP32 division and square root through the hardware rcp/sqrt
             # (about 1 ulp) instead of the correctly rounded sequences; the
             # FP64 path is unaffected
             "-fno-hip-fp32-correctly-rounded-divide-sqrt",
             # FP32 denormals flushed (depths below eps are dry anyway)
             "-fgpu-flush-denormals-to-zero",
             # multiply-adds fused only within one source expression, so
             # that the same expression rounds the same wherever it is
             # inlined (results independent of the tiling of the mesh)
             "-ffp-contract=on",
             "-Wno-unused-result"] + os.environ.get("SWE_EXTRA_HIPFLAGS", "").split()

# per source: the network (in its own kernel and in the stage kernel that
# evaluates it) keeps MFMA accumulators in ordinary vector registers (no
# moves out of accumulation registers between layers)
FILE_FLAGS = {"swe_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
              "swe_device.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True, out: str = LIB, flags=None) -> str:
    hip_flags = HIP_FLAGS if flags is None else flags
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    objs = []
    for src in ("swe_host.cpp", "swe_layers.cpp"):
        obj = os.path.join(HERE, "_build", src.replace(".cpp", ".o"))
        run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-Wall", "-c",
             os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in ("swe_device.hip", "swe_mlp.hip"):
        o = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
        run([HIPCC] + hip_flags + FILE_FLAGS.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = out + f".tmp{os.getpid()}"
    run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
