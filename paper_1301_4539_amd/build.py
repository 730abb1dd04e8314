"""Build libfdtd.so (HIP kernels + C ABI runtime) for gfx950 with hipcc.

Flags that the bit-exactness contract depends on:
  -ffp-contract=off                  no implicit multiply-add fusion (every
                                     fused multiply-add is written explicitly)
  -fno-gpu-flush-denormals-to-zero   keep FP32 subnormals
  -target-feature -packed-fp32-ops   no packed FP32 instructions
and one for speed:
  -falign-loops=64                   loop heads on 64-byte boundaries (the fused
                                     kernel's z-march loops run ~1% faster)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfdtd.so")
SOURCES = ["yee_fused_f32.hip", "yee_fused_f16.hip", "yee_fused_bf16.hip", "yee_fused_graded.hip", "yee_fused_cpml.hip",
           "yee_fused_energy_f32.hip", "yee_fused_energy_f16.hip", "yee_fused_energy_bf16.hip",
           "yee_fused_graded_f16.hip", "yee_fused_graded_bf16.hip", "fdtd_runtime.cpp", "yee_plain.hip",
           "yee_fused.hip", "yee_diag.hip"]


def hipcc_flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-falign-loops=64", "-Wall", "-Wno-unused-result", "-Wno-unknown-pragmas",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, jobs: int = 8) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc] + hipcc_flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _wait(procs):
    bad = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if text.strip():
            print(text, flush=True)
        if p.returncode != 0:
            bad.append(src)
    if bad:
        raise RuntimeError("hipcc failed for " + ", ".join(bad))


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
