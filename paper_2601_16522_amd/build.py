"""Build libpf.so (gfx950 HIP kernels + host engine + C-ABI) in-tree with hipcc.

The fused stage kernels are instantiated once per supported number of order
parameters and number of buffer groups (pf_stage_inst.hip with -DPF_NPHI=n
-DPF_NG=g); those objects compile in parallel and are linked with the
reduction kernels and the host engine.

Two debug builds come with it:
  libpf_poison.so  the same library for N in POISON_NPHI and buffer groups in
                   POISON_NG, with every LDS region filled with NaN before the
                   kernels write it (-DPF_POISON_LDS), so that a read of an
                   element no thread wrote shows up as NaN in the results;
  pf_host_check    a program that calls every C-ABI entry point with exactly
                   sized heap arrays and invalid arguments, linked with the host
                   engine compiled under AddressSanitizer (host code only).
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
LIB_POISON = os.path.join(HERE, "libpf_poison.so")
POISON_NPHI = [2, 4, 9]
POISON_NG = [1, 2]
HOST_CHECK = os.path.join(HERE, "pf_host_check")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

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


def _list_macro(name, values):
    return f"-D{name}(X)=" + " ".join(f"X({v})" for v in values)


def _units():
    units = [(os.path.join(CSRC, "pf_stage_inst.hip"), os.path.join(OBJ, f"stage_n{n}_g{g}.o"),
              [f"-DPF_NPHI={n}", f"-DPF_NG={g}"]) for n in NPHI for g in NGROUPS]
    units.append((os.path.join(CSRC, "pf_kernels.hip"), os.path.join(OBJ, "kernels.o"), []))
    units.append((os.path.join(CSRC, "pf_api.cpp"), os.path.join(OBJ, "api.o"), []))
    return units


def _poison_units():
    pdir = os.path.join(OBJ, "poison")
    units = [(os.path.join(CSRC, "pf_stage_inst.hip"), os.path.join(pdir, f"stage_n{n}_g{g}.o"),
              ["-DPF_POISON_LDS", f"-DPF_NPHI={n}", f"-DPF_NG={g}"])
             for n in POISON_NPHI for g in POISON_NG]
    units.append((os.path.join(CSRC, "pf_kernels.hip"), os.path.join(pdir, "kernels.o"),
                  ["-DPF_POISON_LDS", _list_macro("PF_NPHI_LIST", POISON_NPHI),
                   _list_macro("PF_NG_LIST", POISON_NG)]))
    return units


# AddressSanitizer on the host code only (the device code of these two units
# is the ordinary build)
ASAN = ["-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer", "-g", "-O1"]


def _check_units():
    return [(os.path.join(CSRC, "pf_api.cpp"), os.path.join(OBJ, "asan", "api.o"), ASAN),
            (os.path.join(CSRC, "pf_host_check.cpp"), os.path.join(OBJ, "asan", "pf_host_check.o"),
             ASAN + ["-I" + INCLUDE])]


def build(verbose: bool = False, jobs: int = 0) -> str:
    for d in ("", "poison", "asan"):
        os.makedirs(os.path.join(OBJ, d), exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{r.stderr}")

    def compile_one(u):
        src, obj, extra = u
        # the debug units override the optimisation level after the common flags
        run([HIPCC] + FLAGS + extra + ["-c", src, "-o", obj])
        return obj

    main, poison, check = _units(), _poison_units(), _check_units()

    def cost(u):  # stage units take longest, growing with N: start those first
        n = [int(x.split("=")[1]) for x in u[2] if x.startswith(("-DPF_NPHI=", "-DPF_NG="))]
        return -(100 * n[0] + n[1]) if n else 0

    order = sorted(main + poison + check, key=cost)
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(compile_one, order))
    objs = [u[1] for u in main]

    def link(out, objects, extra=()):
        tmp = out + ".tmp"
        run([HIPCC, "--offload-arch=" + ARCH, *extra, "-o", tmp] + objects)
        os.replace(tmp, out)

    link(LIB, objs, ["-shared", "-fPIC"])
    link(LIB_POISON, [u[1] for u in poison] + [os.path.join(OBJ, "api.o")], ["-shared", "-fPIC"])
    link(HOST_CHECK, [u[1] for u in check] + [o for o in objs if not o.endswith("api.o")],
         ["-Xarch_host", "-fsanitize=address"])
    # the streaming-bandwidth reference program (a measurement aid, not linked)
    run([HIPCC] + FLAGS + [os.path.join(CSRC, "stream_ref.hip"), "-o", STREAM_REF + ".tmp"])
    os.replace(STREAM_REF + ".tmp", STREAM_REF)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
