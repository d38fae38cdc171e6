"""Benchmark of the explicit phase-field + concentration time step on one MI355X.

Default workload: the 1024^2 periodic Voronoi microstructure with 8 order
parameters and c (200 grains, round-robin onto 8 fields, interface parameter
W = 5 cells, c = 0.3 + N(0, 0.01^2)), integrated with adaptive RKL2 (error
estimate and PID controller of Sec. 3.3, a_phi = 1e-2, r = a_c = 1e-4) from
t = 0 to t_end = 100 in the chosen FP32 form.  One benchmark step is one whole
time-to-solution run: every stage kernel (RHS + stage combination + simplex),
the first-stage RHS correction, the estimator with its FP64 reduction, the
controller and the FP64 conservation sum.  The initial state is copied into the
handle (device to device, untimed) before each step.

Prints one JSON line (metric of the project: Gcell-stage/s, i.e. cells x RHS
evaluations per second, with the time to solution and the HBM roofline of the
dominant kernel, the RKL2 inner stage).

Other modes: --workload pores3d (3D grains + pores, fixed RKL2 steps) for the
3D kernel, --copy-calib for the rocprofv3 counter calibration copy kernel.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-solution at fixed sharp-interface error; Gcell-stage/s; % peak HBM GB/s"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2601_16522_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_hash() -> str:
    """Hash of the device sources (any edit invalidates the stored counters)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when they are missing or were taken on another version of the kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(key)
    if not ent or ent.get("kernel_sha") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def make_workload(name: str, size: int):
    import pf_inputs as pi
    if name == "voronoi2d":
        return pi.voronoi_2d(n=size or 1024)
    if name == "pores3d":
        n = size or 256
        return pi.grains_pores_3d(n=n, n_grains=12, n_grain_fields=12, n_pores=40,
                                  r_range=(4.0, 10.0))
    if name == "gg3d":
        n = size or 512
        return pi.grain_growth_pores_3d(n=n)
    raise SystemExit(f"unknown workload {name}")


def copy_calibration(mib: int, reps: int):
    """Plain device copy of known size (for scaling FETCH_SIZE/WRITE_SIZE)."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 4 * n, "reps": reps}), flush=True)


def copy_bandwidth(gib: int = 4, reps: int = 5) -> float:
    """Streaming device-to-device copy of `gib` GiB (read + write counted), GB/s:
    the practical HBM ceiling to set the stencil kernels against."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n / (ms / 1e3) / 1e9


def cpu_baseline(wl, integ: str, t_end: float, tol_kw: dict, dt_fixed: float, sample_note: str):
    """Time the FP64 CPU oracle (as it stands) on the same workload."""
    import oracle
    oracle.build(force=False)
    P = oracle.Params(**wl.param_dict())
    tol = oracle.Tol(**tol_kw) if tol_kw else None
    code = {"rkl2": oracle.RKL2, "fe": oracle.FE, "rkl1": oracle.RKL1}[integ]
    t0 = time.perf_counter()
    u, st, rc = oracle.run_to(P, code, wl.u0, t_end, tol=tol, dt_fixed=dt_fixed)
    el = time.perf_counter() - t0
    cores = oracle.num_threads()
    return {"value": wl.cells * st.rhs_evals / el / 1e9, "unit": "Gcell-stage/s", "cores": cores,
            "kind": "oracle", "sample": sample_note + f"; {st.rhs_evals} RHS evaluations in "
            f"{el:.1f} s, FP64, {cores} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="voronoi2d", choices=["voronoi2d", "pores3d", "gg3d"])
    ap.add_argument("--size", type=int, default=0)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU domain decomposition "
              "is a design (z-slab halos over RCCL), not part of this benchmark", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calib:
        copy_calibration(args.copy_calib, max(args.steps, 1))
        return

    import paper_2601_16522_amd as pf

    t_gen = time.perf_counter()
    wl = make_workload(args.workload, args.size)
    t_gen = time.perf_counter() - t_gen
    print(f"# workload {wl.name}: {wl.cells} cells, {wl.F} fields, generated in {t_gen:.1f} s",
          file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    sim = pf.Sim(wl.param_dict(), prec=args.prec)
    sim.set_stream(stream)
    u0_dev = torch.from_numpy(wl.u0).to(device="cuda", dtype=sim.torch_dtype).contiguous()
    torch.cuda.synchronize()
    dte = sim.stable_dt()

    if args.workload == "voronoi2d":
        integ, t_end, dt_fixed = "rkl2", 100.0, 0.0
        tol_kw = dict(r_phi=1e-4, a_phi=1e-2, r_c=1e-4, a_c=1e-4)
        tol = pf.Tol(**tol_kw)
        desc = "adaptive RKL2 t=0..100, a_phi=1e-2, r=a_c=1e-4"
    else:
        integ, tol_kw, tol = "rkl2", None, None
        dt_fixed = 100.0 * dte
        t_end = 2 * dt_fixed
        desc = "fixed RKL2 at 100 dt_e (21 stages), 2 steps"

    sim.init_fields_device(u0_dev)
    tiling = sim.get_tiling()
    if not args.no_autotune:
        tiling = sim.autotune()[:2]
    print(f"# tiling tx={tiling[0]} zchunk={tiling[1]}", file=sys.stderr, flush=True)

    def one_step():
        sim.init_fields_device(u0_dev)
        stream.synchronize()
        t0 = time.perf_counter()
        st = sim.run_to(integ, t_end, tol=tol, dt_fixed=dt_fixed)
        sim.conservation()
        stream.synchronize()
        return time.perf_counter() - t0, st

    for _ in range(args.warmup):
        one_step()
    sim.set_timing(True)
    torch.cuda.synchronize()
    total, rhs, acc, rej = 0.0, 0, 0, 0
    for k in range(args.steps):
        el, st = one_step()
        total += el
        rhs += st.rhs_evals
        acc += st.accepted
        rej += st.rejected
        print(f"# step {k}: {el * 1e3:.2f} ms, {st.rhs_evals} RHS, {st.accepted} accepted, "
              f"{st.rejected} rejected", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms_rkl2, n_rkl2 = sim.kernel_time(pf.FAM_RKL2)
    ms_stage, n_stage = sim.kernel_time(pf.FAM_STAGE)
    ms_est, n_est = sim.kernel_time(pf.FAM_EST)
    sim.set_timing(False)
    diag = sim.diagnostics()

    copy_bw = copy_bandwidth()
    value = wl.cells * rhs / total / 1e9
    E = 8 if args.prec == "fp64" else 4
    bytes_per_launch = 5 * wl.F * E * wl.cells      # Y_{j-1}, Y_{j-2}, Y_0, R_0 in; Y_j out
    avg_s = ms_rkl2 / max(n_rkl2, 1) / 1e3
    achieved = bytes_per_launch / avg_s / 1e9 if n_rkl2 else 0.0
    key = f"rkl2_stage/{wl.name}/{args.prec}"
    traffic = measured_traffic(key)
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gcell-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {desc}", "cells": wl.cells, "fields": wl.F,
                   "integrator": integ + ("-adaptive" if tol else "-fixed"),
                   "precision": args.prec, "tiling": {"tx": tiling[0], "zchunk": tiling[1]},
                   "rhs_evals_per_step": rhs / args.steps,
                   "accepted_per_step": acc / args.steps, "rejected_per_step": rej / args.steps,
                   "time_to_solution_ms": round(total / args.steps * 1e3, 4),
                   "stage_kernel_ms_per_step": round(ms_stage / args.steps, 4),
                   "estimator_ms_per_step": round(ms_est / args.steps, 4),
                   "max_sum_dev": diag["max_sum_dev"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": f"rkl2_stage_kernel (RKL2 stages j >= 2), {n_rkl2} launches, "
                               f"avg {avg_s * 1e6:.2f} us (HIP events), "
                               f"{bytes_per_launch} algorithmic B/launch",
                     "copy_ref_GBs": round(copy_bw, 1)},
    }
    if not args.no_cpu_baseline:
        note = f"full {wl.name} solve ({desc}) on the host CPU"
        if args.workload != "voronoi2d":
            note = f"one fixed RKL2 step of {wl.name}"
            t_end_cpu = dt_fixed
        else:
            t_end_cpu = t_end
        out["cpu_baseline"] = cpu_baseline(wl, integ, t_end_cpu, tol_kw, dt_fixed, note)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
