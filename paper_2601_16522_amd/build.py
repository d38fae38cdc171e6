"""Build libpf.so (gfx950 HIP kernels + host engine + C-ABI) in-tree with hipcc.

The fused stage kernels are instantiated once per supported number of order
parameters and number of buffer groups (pf_stage_inst.hip with -DPF_NPHI=n
-DPF_NG=g); those objects compile in parallel and are linked with the
reduction kernels and the host engine.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpf.so")
STREAM_REF = os.path.join(HERE, "stream_ref")
NPHI = [2, 3, 4, 8, 9, 13]
NGROUPS = [1, 2, 4]  # buffer groups per state vector (kernels are compiled per count)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # fixed IEEE evaluation order (no fused multiply-add contraction)
    "-ffp-contract=off",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-Wno-unused-value", "-Wno-unused-result",
]


def _units():
    units = [(os.path.join(CSRC, "pf_stage_inst.hip"), os.path.join(OBJ, f"stage_n{n}_g{g}.o"),
              [f"-DPF_NPHI={n}", f"-DPF_NG={g}"]) for n in NPHI for g in NGROUPS]
    units.append((os.path.join(CSRC, "pf_kernels.hip"), os.path.join(OBJ, "kernels.o"), []))
    units.append((os.path.join(CSRC, "pf_api.cpp"), os.path.join(OBJ, "api.o"), []))
    return units


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)

    def compile_one(u):
        src, obj, extra = u
        cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, _units()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # the streaming-bandwidth reference program (a measurement aid, not linked)
    cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, "stream_ref.hip"), "-o", STREAM_REF + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(STREAM_REF + ".tmp", STREAM_REF)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
