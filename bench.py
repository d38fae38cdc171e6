"""Benchmark of the explicit phase-field + concentration time step on one MI355X.

Default workload: 3D periodic grain growth with pores at 512^3 (2000 seeded
Voronoi grains round-robin onto 8 order parameters, a pore phase of 400
seeded spheres of radius 3-8 cells, c = 1 in the pores and 0 in the solid;
the paper's mobile-pore parameter set of Sec. 5.3), ten fixed RKL2 steps of
100 dt_e (21 stages each, eq. sts with the five-vector storage) to
t_end = 1000 dt_e in the chosen FP32 form, with the FP64 conservation sum at
the end.  One benchmark step is that whole run: every stage kernel (RHS +
stage combination + simplex projection), the first-stage RHS correction and
the FP64 sum of c.  The initial state is copied into the handle (device to
device, untimed) before each step.

Prints one JSON line: Gcell-stage/s (cells x RHS evaluations per second), the
time to solution, the HBM roofline of the dominant kernel (the RKL2 inner
stage), the FP64 oracle timed on the host on a bounded sample of the same
workload, and, under config.batch_equal_error, the comparison at equal
sharp-interface error: 96 uneven 2D shrinking grains batched in FP32
against the plain FP64 form instance by instance.

Other modes: --workload pores3d (256^3 sintering, two fixed RKL2 steps; with
--adaptive, adaptive RKL2 to t_end = 1e-3), --workload voronoi2d (the
1024^2 eight-field microstructure, adaptive RKL2 to t = 100; its 189 MB
footprint is resident in the 256 MB last-level cache), --workload batch (the
96-instance batch with its RKL2 and adaptive legs), --copy-calib for the
rocprofv3 counter calibration copy kernel.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math

import numpy as np
import os
import subprocess
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
        if name.endswith((".hip", ".hpp", ".h")) and name != "stream_ref.hip":
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


def stream_reference(vector_bytes: int, planes=None):
    """Streaming references at the stage's own footprint: the committed
    stream_ref program (built beside the library) run as a child process on
    vectors of `vector_bytes` bytes.  Returns GB/s of its 4-read-1-write,
    copy and read-only kernels, and with planes = (F, nx, ny) also of the
    stage kernels' own access pattern (F planes per vector, 64 x 4 tiles
    marched in z), or None when the program is not built."""
    exe = os.path.join(ROOT, "paper_2601_16522_amd", "stream_ref")
    if not os.path.exists(exe):
        return None
    n = max(1024, vector_bytes // 4)
    extra = [str(v) for v in planes] if planes else []
    r = subprocess.run([exe, str(n), "10", *extra], capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        print(f"# stream_ref failed: {r.stderr.strip()}", file=sys.stderr, flush=True)
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def z_slab(wl, planes: int):
    """The first `planes` z planes of a 3D workload as a periodic grid of their
    own: the same fields and value distribution, a bounded sample for timing
    the CPU oracle."""
    import dataclasses
    if wl.dim != 3 or planes >= wl.nz:
        return wl
    u0 = np.ascontiguousarray(wl.u0[:, :planes])
    return dataclasses.replace(wl, name=f"{wl.name}[z<{planes}]", nz=planes, u0=u0)


def cpu_baseline(wl, integ: str, t_end: float, tol_kw: dict, dt_fixed: float, sample_note: str):
    """Time the FP64 CPU oracle (as it stands) on a workload."""
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


def area_slope_error(u0, u, t, M, dx=1.0, gamma=1.0):
    """Relative error of the mean area rate (A(t) - A(0))/t of the grain
    (phase 1) against the curvature-flow law -2 pi M gamma (Sec. 5.2.1)."""
    rate = (u[1].sum() - u0[1].sum()) * dx * dx / t
    return abs(rate / (-2 * math.pi * M * gamma) - 1.0)


def batch_equal_error():
    """The comparison at equal sharp-interface error: the 96
    shrinking-grain instances, 2000 forward-Euler steps each at 0.9 dt_e,
    batched in FP32 (one fused launch per step, autotuned, hipGraphs of 50
    launches) against the plain FP64 form run instance by instance; the error
    is that of the mean area rate against dA/dt = -2 pi M gamma (Sec. 5.2.1).
    One untimed run each to warm up, then one timed run each."""
    import torch
    import paper_2601_16522_amd as pf
    import pf_inputs as pi
    nsteps = 2000
    wls = pi.batch_instances()
    stream = torch.cuda.Stream()
    b = pf.Batch([w.param_dict() for w in wls], prec="fp32")
    b.set_stream(stream)
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    dts = [0.9 * b.stable_dt(i) for i in range(len(wls))]
    t_end = [nsteps * d for d in dts]
    b.autotune()

    def run32():
        for i, w in enumerate(wls):
            b.init_fields(i, w.u0)
        stream.synchronize()
        t0 = time.perf_counter()
        b.run_to(t_end, dt=dts, graph_steps=50)
        stream.synchronize()
        return time.perf_counter() - t0

    run32()
    t32 = run32()
    err32 = [area_slope_error(w.u0, b.get_fields(i)[0], t_end[i], w.mob[0]) for i, w in enumerate(wls)]
    b.close()
    t64, err64 = 0.0, []
    for i, w in enumerate(wls):
        s = pf.Sim(w.param_dict(), prec="fp64")
        s.set_stream(stream)
        for rep in range(2 if i == 0 else 1):  # the first instance once more, to warm up
            s.init_fields(w.u0)
            stream.synchronize()
            ts = time.perf_counter()
            s.run_to("fe", t_end[i], dt_fixed=dts[i])
            stream.synchronize()
        t64 += time.perf_counter() - ts
        err64.append(area_slope_error(w.u0, s.get_fields()[0], t_end[i], w.mob[0]))
        s.close()
    return {"workload": f"{len(wls)} 2D shrinking grains (side 64..512, R 0.2..0.4 side, "
                        f"M 0.5..2), {sum(w.cells for w in wls)} cells, {nsteps} FE steps each "
                        f"at 0.9 dt_e",
            "fp32_batched_ms": round(t32 * 1e3, 3), "fp64_per_instance_ms": round(t64 * 1e3, 3),
            "speedup": round(t64 / t32, 2),
            "area_rate_rel_error_fp32_batched": float(np.mean(err32)),
            "area_rate_rel_error_fp64_per_instance": float(np.mean(err64)),
            "area_rate_rel_error_max_abs_diff": float(np.max(np.abs(np.subtract(err32, err64))))}


def batch_bench(args):
    """96 independent shrinking-grain instances (side 64..512 by seed, R in
    [0.2, 0.4] side, M in [0.5, 2]): 2000 forward-Euler steps each at 0.9 dt_e,
    as one fused launch per step replayed from a hipGraph in FP32, against the
    plain FP64 form run instance by instance; then the same end times with
    batched RKL2 steps of --rkl2-dte dt_e, and with adaptive batched RKL2
    (a controller per instance, the tolerances of the 1024^2 Voronoi run)."""
    import torch
    import paper_2601_16522_amd as pf
    import pf_inputs as pi
    nsteps = 2000
    wls = pi.batch_instances()
    cells = sum(w.cells for w in wls)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    b = pf.Batch([w.param_dict() for w in wls], prec=args.prec)
    b.set_stream(stream)
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    dts = [0.9 * b.stable_dt(i) for i in range(len(wls))]
    t_end = [nsteps * d for d in dts]
    if not args.no_autotune:
        b.autotune()
    if args.blocks:
        b.set_blocks(args.blocks)
    if args.fusion:
        b.set_fusion(args.fusion)
    nb, depth = b.config()
    K = args.graph_steps

    def one():
        for i, w in enumerate(wls):
            b.init_fields(i, w.u0)
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        b.run_to(t_end, dt=dts, graph_steps=K)
        e1.record(stream)
        stream.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    total, ev_ms = 0.0, 0.0
    for k in range(args.steps):
        el, ms = one()
        total += el
        ev_ms += ms
        print(f"# batch step {k}: {el * 1e3:.2f} ms", file=sys.stderr, flush=True)
    err32 = [area_slope_error(w.u0, b.get_fields(i)[0], t_end[i], w.mob[0]) for i, w in enumerate(wls)]

    # the same end times with batched RKL2 steps of args.rkl2_dte dt_e (eq. sts)
    dts_rkl2 = [args.rkl2_dte / 0.9 * d for d in dts]
    rkl2_ms, rkl2_rhs = [], 0
    for k in range(max(args.steps, 1) + 1):
        for i, w in enumerate(wls):
            b.init_fields(i, w.u0)
        stream.synchronize()
        t0 = time.perf_counter()
        st_r = b.run_to(t_end, dt=dts_rkl2, graph_steps=10, integ="rkl2")
        stream.synchronize()
        if k > 0:  # the first run captures the graph
            rkl2_ms.append((time.perf_counter() - t0) * 1e3)
        rkl2_rhs = sum(x.rhs_evals for x in st_r)
    err_rkl2 = [area_slope_error(w.u0, b.get_fields(i)[0], t_end[i], w.mob[0]) for i, w in enumerate(wls)]

    # the same end times with adaptive RKL2, one controller per instance (Sec. 3.3)
    tol = pf.Tol(r_phi=1e-4, a_phi=1e-2, r_c=1e-4, a_c=1e-4)
    ad_ms, st_a = [], []
    for k in range(max(args.steps, 1) + 1):
        for i, w in enumerate(wls):
            b.init_fields(i, w.u0)
        stream.synchronize()
        t0 = time.perf_counter()
        st_a = b.run_adaptive(t_end, tol)
        stream.synchronize()
        if k > 0:  # the first run allocates the adaptive buffers
            ad_ms.append((time.perf_counter() - t0) * 1e3)
    err_ad = [area_slope_error(w.u0, b.get_fields(i)[0], t_end[i], w.mob[0]) for i, w in enumerate(wls)]

    # the plain FP64 form, instance by instance (one launch per step each)
    t64 = 0.0
    err64 = []
    for i, w in enumerate(wls if not args.no_fp64_ref else []):
        s = pf.Sim(w.param_dict(), prec="fp64")
        s.set_stream(stream)
        s.init_fields(w.u0)
        stream.synchronize()
        ts = time.perf_counter()
        s.run_to("fe", t_end[i], dt_fixed=dts[i])
        stream.synchronize()
        t64 += time.perf_counter() - ts  # the runs only, not the uploads
        err64.append(area_slope_error(w.u0, s.get_fields()[0], t_end[i], w.mob[0]))
        s.close()
    value = cells * nsteps / (total / args.steps) / 1e9
    E = 4 if args.prec == "fp32" else 8
    F = wls[0].F
    # algorithmic bytes: 2 F E per cell and forward-Euler step, times the
    # cell-steps of one launch (depth steps); the fused launch itself reads
    # the state once and writes it once
    bytes_per_launch = 2 * F * E * cells * depth
    min_bytes_per_launch = 2 * F * E * cells
    launches = -(-nsteps // depth)
    avg_s = ev_ms / args.steps / launches / 1e3
    achieved = bytes_per_launch / avg_s / 1e9
    traffic = measured_traffic(f"batch_euler_d{depth}/{len(wls)}inst/{args.prec}")
    sref = stream_reference(F * E * cells)
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gcell-stage/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"batch of {len(wls)} 2D shrinking grains, {cells} cells, "
                               f"{nsteps} FE steps each at 0.9 dt_e, one fused launch per "
                               f"{depth} step(s), "
                               + (f"hipGraphs of {K} launches" if K > 0 else "direct launches"),
                   "cells": cells, "instances": len(wls), "persistent_blocks": nb,
                   "fusion_depth": depth,
                   "state_GBs_per_step": round(2 * F * E * cells / (avg_s / depth) / 1e9, 1),
                   "time_to_solution_ms": round(total / args.steps * 1e3, 3),
                   "area_rate_rel_error_fp32_batch_mean": float(np.mean(err32)),
                   "rkl2_batch": {"step_dt_e": args.rkl2_dte, "rhs_evals": int(rkl2_rhs),
                                  "time_to_solution_ms": round(float(np.mean(rkl2_ms)), 3),
                                  "speedup_vs_fe_batch": round(total / args.steps * 1e3 / float(np.mean(rkl2_ms)), 2),
                                  "area_rate_rel_error_mean": float(np.mean(err_rkl2))},
                   "rkl2_adaptive_batch": {
                       "tol": {"r_phi": tol.r_phi, "a_phi": tol.a_phi, "r_c": tol.r_c, "a_c": tol.a_c},
                       "accepted": int(sum(x.accepted for x in st_a)),
                       "rejected": int(sum(x.rejected for x in st_a)),
                       "rhs_evals": int(sum(x.rhs_evals for x in st_a)),
                       "batch_steps": int(max(x.accepted + x.rejected for x in st_a)),
                       "time_to_solution_ms": round(float(np.mean(ad_ms)), 3),
                       "speedup_vs_fe_batch": round(total / args.steps * 1e3 / float(np.mean(ad_ms)), 2),
                       "area_rate_rel_error_mean": float(np.mean(err_ad))}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": f"batch_kernel (forward Euler, depth {depth}), avg {avg_s * 1e6:.2f} us per launch "
                               f"of {depth} step(s) (HIP events over graph replays), "
                               f"{bytes_per_launch} algorithmic B/launch",
                     "steps_per_launch": depth,
                     "fused_min_bytes_per_launch": min_bytes_per_launch,
                     "frac_of_fused_min": round(min_bytes_per_launch / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                     "stream_ref_GBs": sref,
                     "frac_of_stream_copy": round(achieved / sref["copy"], 4) if sref else None},
    }
    if err64:
        out["config"].update({
            "fp64_per_instance_time_ms": round(t64 * 1e3, 3),
            "speedup_vs_fp64_per_instance": round(t64 / (total / args.steps), 2),
            "area_rate_rel_error_fp64_single_mean": float(np.mean(err64)),
            "area_rate_rel_error_max_abs_diff": float(np.max(np.abs(np.subtract(err32, err64))))})
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gg3d",
                    choices=["voronoi2d", "pores3d", "gg3d", "batch"])
    ap.add_argument("--size", type=int, default=0)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--zchunk", type=int, default=0,
                    help="z planes per block (3D); skips the tiling autotuner")
    ap.add_argument("--pair-zchunk", type=int, default=0,
                    help="z planes per block of the 3D fused RKL2 stage pairs; skips the "
                         "tiling autotuner")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB")
    ap.add_argument("--blocks", type=int, default=0,
                    help="batch: persistent grid size (skips the block-count autotuner)")
    ap.add_argument("--rkl2-dte", type=float, default=50.0,
                    help="batch: RKL2 step in units of dt_e for the RKL2 comparison")
    ap.add_argument("--fusion", type=int, default=0, choices=[0, 1, 2],
                    help="batch: FE steps per launch; single simulations: RKL2 inner stages per "
                         "launch (2: fused pairs, 2D); 0: the autotuner's choice")
    ap.add_argument("--graph-steps", type=int, default=50,
                    help="batch: steps per captured hipGraph (0: direct launches)")
    ap.add_argument("--integ", default="rkl2", choices=["rkl2", "rkl1"],
                    help="pores3d/gg3d fixed steps: RKL2 (5-vector storage) or RKL1 (the "
                         "3-vector ring of Alg. sts1); the roofline then covers all of RKL1's "
                         "stage launches")
    ap.add_argument("--adaptive", action="store_true",
                    help="pores3d: adaptive RKL2 to t_end = 1e-3 with r = a = 1e-4 (the 256^3 "
                         "sintering run) instead of two fixed steps")
    ap.add_argument("--no-fp64-ref", action="store_true",
                    help="batch: skip the FP64 instance-by-instance comparison")
    ap.add_argument("--no-batch-leg", action="store_true",
                    help="skip the batched FP32 against per-instance FP64 comparison of the "
                         "default line")
    ap.add_argument("--sparse", type=int, default=0, metavar="N_P",
                    help="3D fixed steps: sparse phase storage with at most N_P nonzero phases per "
                         "cell (Sec. 3.1); a projected cell with more keeps the N_P largest and the "
                         "line reports how many cells were cut")
    ap.add_argument("--r0-recompute", default="auto", choices=["auto", "0", "1"],
                    help="3D RKL2 inner stages: recompute R0 from u0 (1) or read it (0); auto: the "
                         "autotuner's choice (read it when the autotuner is skipped)")
    ap.add_argument("--cpu-planes", type=int, default=64,
                    help="3D workloads: z planes of the sample the CPU oracle is timed on")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; the multi-GPU domain decomposition "
              "is a design (z-slab halos over RCCL), not part of this benchmark", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calib:
        copy_calibration(args.copy_calib, max(args.steps, 1))
        return

    import paper_2601_16522_amd as pf

    if args.workload == "batch":
        batch_bench(args)
        return

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
    elif args.adaptive and args.workload == "pores3d":
        integ, t_end, dt_fixed = "rkl2", 1e-3, 0.0
        tol_kw = dict(r_phi=1e-4, a_phi=1e-4, r_c=1e-4, a_c=1e-4)
        tol = pf.Tol(**tol_kw)
        desc = "adaptive RKL2 t=0..1e-3, r=a=1e-4"
    elif args.adaptive:
        raise SystemExit("--adaptive applies to --workload pores3d")
    else:
        # 512^3: ten steps of the 5-vector RKL2 scheme (to t = 1000 dt_e); 256^3: two
        integ, tol_kw, tol = args.integ, None, None
        dt_fixed = 100.0 * dte
        nfix = 10 if args.workload == "gg3d" else 2
        t_end = nfix * dt_fixed
        s_fix = pf.rkl_stage_count(integ, dt_fixed, dte)
        desc = f"fixed {integ.upper()} at 100 dt_e ({s_fix} stages), {nfix} steps"
    rkl1 = integ == "rkl1"
    if rkl1 and args.workload not in ("pores3d", "gg3d") or rkl1 and args.adaptive:
        raise SystemExit("--integ rkl1 applies to fixed steps of --workload pores3d|gg3d")

    if args.sparse:
        if wl.dim != 3 or args.adaptive or args.fusion == 2:
            raise SystemExit("--sparse applies to fixed steps of --workload pores3d|gg3d")
        sim.set_sparse_storage(args.sparse)
    sim.init_fields_device(u0_dev)
    tiling = sim.get_tiling()
    if args.zchunk or args.pair_zchunk:
        if args.zchunk:
            sim.set_tiling(tiling[0], args.zchunk)
        if args.pair_zchunk:
            sim.set_pair_zchunk(args.pair_zchunk)
        tiling = sim.get_tiling()
    elif not args.no_autotune and not args.sparse:
        tiling = sim.autotune()[:2]
    if args.fusion:
        sim.set_stage_fusion(args.fusion)
    if args.r0_recompute != "auto":
        sim.set_r0_recompute(args.r0_recompute == "1")
    fusion = sim.get_stage_fusion()
    pair_zc = sim.get_pair_zchunk()
    recompute = sim.get_r0_recompute() and fusion == 1 and not rkl1 and not args.sparse
    print(f"# tiling tx={tiling[0]} zchunk={tiling[1]} pair zchunk={pair_zc}, RKL2 stages per "
          f"launch {fusion}, R0 recomputed {recompute}", file=sys.stderr, flush=True)

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
    # the timed runs record one event pair per step, around the inner RKL2
    # stages only (events between other launches would add gaps to the time
    # to solution)
    fam = pf.FAM_STAGE if rkl1 else pf.FAM_RKL2
    sim.set_timing(True, families=[fam])
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
    ms_rkl2, n_rkl2 = sim.kernel_time(fam)
    # the breakdown by kernel family from one more run, untimed
    sim.set_timing(True)
    one_step()
    ms_stage, n_stage = sim.kernel_time(pf.FAM_STAGE)
    ms_est, n_est = sim.kernel_time(pf.FAM_EST)
    sim.set_timing(False)
    diag = sim.diagnostics()

    E = 8 if args.prec == "fp64" else 4
    sref = stream_reference(wl.F * E * wl.cells, (wl.F, wl.nx, wl.ny) if wl.dim == 3 and E == 4 else None)
    value = wl.cells * rhs / total / 1e9
    cuts = sim.sparse_cuts() if args.sparse else None
    if args.sparse and not rkl1:
        # Y_{j-1}, Y_{j-2}, Y_0 and Y_j in sparse storage (c, N_P phase slots and
        # the id word per cell), R_0 dense
        per_cell = 4 * (args.sparse + (1 if wl.with_c else 0) + 1) + wl.F
        bytes_per_launch = per_cell * E * wl.cells
        key = f"rkl2_stage_sparse{args.sparse}/{wl.name}/{args.prec}"
        kname = (f"rkl2_stage_kernel in sparse storage (N_P = {args.sparse}, RKL2 stages j >= 2), "
                 f"{n_rkl2} launches")
    elif rkl1:
        # stage 1 reads u and writes Y_1; stages j >= 2 read Y_{j-1}, Y_{j-2}, write Y_j
        bytes_per_launch = round((2 + 3 * (s_fix - 1)) / s_fix * wl.F * E * wl.cells)
        key = f"rkl1_stages/{wl.name}/{args.prec}"
        kname = f"rkl1 stages (euler first stage + rkl1_stage_kernel), {n_rkl2} launches"
    elif fusion == 2:
        # two stages per launch: 5 F E per cell and stage times two stages; the
        # fused launch itself reads Y_{j-1}, Y_{j-2}, Y_0, R_0 and writes Y_j,
        # Y_{j+1} once (6 F E per cell)
        bytes_per_launch = 10 * wl.F * E * wl.cells
        key = f"rkl2_pair/{wl.name}/{args.prec}"
        kname = (f"rkl2_pair{'3' if wl.dim == 3 else ''}_kernel (RKL2 stages j, j + 1 fused), "
                 f"{n_rkl2} launches")
    elif recompute:
        # Y_{j-1} and Y_0 (stencils), Y_{j-2} in; Y_j out; R_0 recomputed from Y_0
        bytes_per_launch = 4 * wl.F * E * wl.cells
        key = f"rkl2_stage_rc/{wl.name}/{args.prec}"
        kname = f"rkl2_rc_stage_kernel (RKL2 stages j >= 2, R0 recomputed), {n_rkl2} launches"
    else:
        bytes_per_launch = 5 * wl.F * E * wl.cells      # Y_{j-1}, Y_{j-2}, Y_0, R_0 in; Y_j out
        key = f"rkl2_stage/{wl.name}/{args.prec}"
        kname = f"rkl2_stage_kernel (RKL2 stages j >= 2), {n_rkl2} launches"
    avg_s = ms_rkl2 / max(n_rkl2, 1) / 1e3
    achieved = bytes_per_launch / avg_s / 1e9 if n_rkl2 else 0.0
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
                   "precision": args.prec,
                   "tiling": {"tx": tiling[0], "zchunk": tiling[1], "pair_zchunk": pair_zc},
                   "rkl2_stages_per_launch": fusion,
                   "r0_recomputed": bool(recompute),
                   "rhs_evals_per_step": rhs / args.steps,
                   "accepted_per_step": acc / args.steps, "rejected_per_step": rej / args.steps,
                   "time_to_solution_ms": round(total / args.steps * 1e3, 4),
                   "stage_kernel_ms_per_step": round(ms_stage, 4),
                   "estimator_ms_per_step": round(ms_est, 4),
                   "max_sum_dev": diag["max_sum_dev"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": f"{kname}, avg {avg_s * 1e6:.2f} us (HIP events), "
                               f"{bytes_per_launch} algorithmic B/launch",
                     "stages_per_launch": 2 if (fusion == 2 and not rkl1) else 1,
                     "fused_min_bytes_per_launch": (6 * wl.F * E * wl.cells
                                                    if (fusion == 2 and not rkl1) else bytes_per_launch),
                     "frac_of_fused_min": round((6 * wl.F * E * wl.cells if (fusion == 2 and not rkl1)
                                                 else bytes_per_launch) / max(avg_s, 1e-12) / 1e9
                                                / HBM_PEAK_GBS, 4),
                     "us_per_stage": round(avg_s * 1e6 / (2 if (fusion == 2 and not rkl1) else 1), 3),
                     "stream_ref_GBs": sref,
                     "frac_of_stream_4r1w": round(achieved / sref["4r1w"], 4) if sref else None,
                     "frac_of_stream_4r1w_planes": (round(achieved / sref["4r1w_planes"], 4)
                                                    if sref and "4r1w_planes" in sref else None)},
    }
    if args.sparse:
        # cells cut by the storage rule over every run of this process (warm-up,
        # timed and the untimed breakdown run)
        out["config"]["sparse_storage"] = {"n_p": args.sparse, "cells_cut": cuts,
                                           "runs": args.warmup + args.steps + 1,
                                           "dense_bytes_per_launch": 5 * wl.F * E * wl.cells}
    if args.workload == "gg3d" and not args.no_batch_leg:
        print("# batch leg: FP32 batched against FP64 per instance", file=sys.stderr, flush=True)
        out["config"]["batch_equal_error"] = batch_equal_error()
    if not args.no_cpu_baseline:
        note = f"full {wl.name} solve ({desc}) on the host CPU"
        cwl = wl
        if args.workload != "voronoi2d":
            # a bounded sample: one fixed step at 100 dt_e (the same stage count
            # and mix) on the first z planes of the same state, periodic in z
            cwl = z_slab(wl, args.cpu_planes)
            note = (f"one fixed {args.integ.upper()} step at 100 dt_e "
                    f"({pf.rkl_stage_count(args.integ, 100.0 * dte, dte)} stages) on {cwl.name}, "
                    f"{cwl.cells} cells (the first {cwl.nz} z planes of the same state, periodic)")
            dt_fixed = 100.0 * dte
            integ, tol_kw = args.integ, None
            t_end_cpu = dt_fixed
        else:
            t_end_cpu = t_end
        print(f"# cpu baseline: {note}", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cwl, integ, t_end_cpu, tol_kw, dt_fixed, note)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
