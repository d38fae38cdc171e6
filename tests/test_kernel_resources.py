"""Compile-time resource checks of the gfx950 stage kernels (CPU only).

Every stage kernel keeps its state in registers and LDS: a kernel that spills
to per-lane scratch runs an order of magnitude slower without any change in
its results, so no parity test would notice.  The check compiles the stage
instantiations for the order-parameter counts of the measured workloads
(N = 8: the 2D Voronoi case; N = 13: the largest, 3D grains + pores) and reads
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


def _resource_remarks(nphi, tmp_path):
    import build as pfbuild  # the package's build script: its flags are the product's

    src = os.path.join(ROOT, "paper_2601_16522_amd", "csrc", "pf_stage_inst.hip")
    cmd = [HIPCC, *pfbuild.FLAGS, f"-DPF_NPHI={nphi}", "-c", src, "-o",
           str(tmp_path / f"s{nphi}.o"), "--offload-device-only",
           "-Rpass-analysis=kernel-resource-usage"]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stderr[-2000:]
    kernels, name = {}, None
    for line in p.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.search(r"remark:\s+(ScratchSize \[bytes/lane\]|VGPRs|AGPRs|Occupancy \[waves/SIMD\]): (\d+)",
                      line)
        if m and name:
            kernels[name][m.group(1)] = int(m.group(2))
    return kernels


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_stage_kernels_do_not_spill(tmp_path):
    with ThreadPoolExecutor(2) as ex:
        res = list(ex.map(lambda n: (n, _resource_remarks(n, tmp_path)), (8, 13)))
    for n, kernels in res:
        # nine stage kinds x {float, double} x {2D, 3D} plus the batch kernel
        names = [k for k in kernels if "_kernel" in k]
        assert len(names) >= 9 * 2 * 2 + 2, (n, sorted(kernels))
        for k in names:
            assert kernels[k].get("ScratchSize [bytes/lane]", 0) == 0, (n, k, kernels[k])
        # batch kernels: depth 1 in both precisions, depth 2 where its LDS fits
        # (FP32 for every N, FP64 only up to N = 4)
        batch = [k for k in names if "batch_euler_kernel" in k]
        assert len(batch) == 3, batch
