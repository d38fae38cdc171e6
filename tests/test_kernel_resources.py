"""Compile-time resource checks of the gfx950 stage kernels (CPU only).

Every stage kernel keeps its state in registers and LDS: a kernel that spills
to per-lane scratch runs an order of magnitude slower without any change in
its results, so no parity test would notice; single-precision kernels must not
spill scalar registers either (each reload is a vector instruction).  The
check compiles the stage instantiations of the measured workloads and reads
the compiler's resource-usage remarks.
"""

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2601_16522_amd"))

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _resource_remarks(nphi, ngroups, tmp_path):
    import build as pfbuild  # the package's build script: its flags are the product's

    src = os.path.join(ROOT, "paper_2601_16522_amd", "csrc", "pf_stage_inst.hip")
    cmd = [HIPCC, *pfbuild.FLAGS, f"-DPF_NPHI={nphi}", f"-DPF_NG={ngroups}", "-c", src, "-o",
           str(tmp_path / f"s{nphi}_{ngroups}.o"), "--offload-device-only",
           "-Rpass-analysis=kernel-resource-usage"]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert p.returncode == 0, p.stderr[-2000:]
    kernels, name = {}, None
    for line in p.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.search(r"remark:\s+(ScratchSize \[bytes/lane\]|VGPRs|AGPRs|SGPRs Spill|VGPRs Spill|"
                      r"Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and name:
            kernels[name][m.group(1)] = int(m.group(2))
    return kernels


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_stage_kernels_do_not_spill(tmp_path):
    """(N, buffer groups) of the measured workloads: 2D Voronoi (8, 1), 512^3
    grain growth in FP32 (9, 2), 256^3 grains + pores (13, 1)."""
    units = [(8, 1), (9, 2), (13, 1)]
    with ThreadPoolExecutor(3) as ex:
        res = list(ex.map(lambda u: (u, _resource_remarks(u[0], u[1], tmp_path)), units))
    for (n, g), kernels in res:
        # nine stage kinds x {float, double} x {2D, 3D}, plus the batch kernels
        names = [k for k in kernels if "_kernel" in k]
        assert len(names) >= 9 * 2 * 2, (n, g, sorted(kernels))
        for k in names:
            r = kernels[k]
            assert r.get("ScratchSize [bytes/lane]", 0) == 0, (n, g, k, r)
            assert r.get("VGPRs Spill", 0) == 0, (n, g, k, r)
            # single precision: no SGPR spills either, except in the 3D fused
            # stage pair (an autotuner candidate, off by default), whose six
            # vectors' buffer descriptors per group fill the scalar file, and
            # in the sparse-storage instances (last template flag set), which
            # add the id-word bases of four vectors: a few spill into vector
            # lanes (never to memory)
            sparse = "Lb1EEEvNS" in k
            if "IfLi" in k and "rkl2_pair3_kernel" not in k and not sparse:
                assert r.get("SGPRs Spill", 0) == 0, (n, g, k, r)
        # batch kernels (built with one group), per precision: forward Euler at
        # depth 1, the two RKL2 stage kinds, the error estimate, and forward
        # Euler at depth 2 where it is built
        # sparse phase storage: RHS, Euler, RKL1 and both RKL2 stage kinds
        # x {float, double} x {2D, 3D}, for one and two buffer groups
        sp = [k for k in names if "Lb1EEEvNS" in k]
        assert len(sp) == (5 * 2 * 2 if g <= 2 else 0), (n, g, sorted(sp))
        batch = [k for k in names if "batch_kernel" in k]
        expect = 8 + sum(_depth2_fits(esz, n) for esz in (4, 8))
        assert len(batch) == (expect if g == 1 else 0), (n, g, batch)
        # 3D stages that recompute R0: single precision N <= 9, double N <= 4
        # (two z windows per thread within two waves per SIMD, no scratch)
        rc = [k for k in names if "rkl2_rc_stage_kernel" in k]
        assert len(rc) == int(n <= 9) + int(n <= 4), (n, g, rc)
        # fused RKL2 stage pairs: one group, where the LDS fits; 512-thread
        # blocks, two per CU by LDS, so four waves per SIMD need <= 128 VGPRs
        pairs = [k for k in names if "rkl2_pair_kernel" in k]
        expect = sum(_pair_fits(esz, n) for esz in (4, 8))
        assert len(pairs) == (expect if g == 1 else 0), (n, g, pairs)
        for k in pairs:
            assert kernels[k].get("VGPRs", 999) <= 128, (n, g, k, kernels[k])


def _pair_fits(esz, n):
    """The LDS rule of the fused RKL2 stage-pair kernel (pf_internal.h)."""
    txt = open(os.path.join(ROOT, "paper_2601_16522_amd", "csrc", "pf_internal.h")).read()
    m = re.search(r"constexpr int P2_TX = (\d+), P2_TY = (\d+), P2_THREADS = P2_TX \* P2_TY, "
                  r"P2_LDS_MAX = (\d+);", txt)
    tx, ty, cap = (int(g) for g in m.groups())
    lds = (n + 3) * (tx + 4) * (ty + 4) + (n + 2) * (tx + 2) * (ty + 2) + 3 * n * n + 4 * n
    return esz * lds <= cap


def _depth2_fits(esz, n):
    """The LDS rule of the fused two-step batch kernel (pf_internal.h)."""
    txt = open(os.path.join(ROOT, "paper_2601_16522_amd", "csrc", "pf_internal.h")).read()
    if n > int(re.search(r"constexpr int DEPTH2_MAX_N = (\d+);", txt).group(1)):
        return False
    rows = 2 if n <= int(re.search(r"constexpr int ROWS2D_MAX_N = (\d+);", txt).group(1)) else 1
    ty = 4 * rows
    f2 = 68 * (ty + 4) + 66 * (ty + 2)
    return esz * ((n + 3) * f2 + 3 * n * n + 4 * n) <= 65536
