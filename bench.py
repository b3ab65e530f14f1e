"""Benchmark: Riccati trajectory-steps/s of full self-consistency iterations.

One step = one Picard iteration of the whole hot path on one GPU:
interpolation onto the rotated lattices, gamma / gamma~ sweeps with the
Green's functions and pole sums, rotate-back with the gap / current / free
energy update, the A-solve, residuals and the Picard update.  Workload: the
400x400 d-wave square with [110] edges (side 40 xi0, h = 0.1), 64 angles,
64 Ozaki poles, t = 0.1, one flux quantum, kappa = 20, one seeded vortex.
Inputs are resident in HBM before the timed region.  The reported value is
the mixed FP32-sweep / FP64-sum path; the FP64 path is timed beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "Riccati trajectory-steps/s, FP32-mixed vs FP64 at 1e-4*Delta0 error; %roofline"
WORKLOAD = "d110_square_400"
# algorithmic flops (complex ops expanded into real ones; sqrt, reciprocal
# count one each): per implicit-midpoint step (App. C) and per node and pole
# for the Green's functions and the three pole sums
FLOPS_PER_STEP = 71
FLOPS_PER_NODE_POLE = 82
PEAK_VALU_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, FP64 and unpacked FP32
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# HBM bytes per sweep launch (mixed) from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs scaled by a plain-copy calibration (profiles/sweep_kernel_d110_square_400.md);
# None whenever the kernel changed after the counters were taken.
SWEEP_TRAFFIC_BYTES = 11.40e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-angles", type=int, default=4)
    ap.add_argument("--skip-fp64", action="store_true")
    return ap.parse_args()


def timed_scf(qs, torch, sp, precision, d0, a0, steps, warmup):
    g = qs.Grain(sp, precision)
    dd = torch.as_tensor(d0).cuda()
    ad = torch.as_tensor(a0).cuda()
    if warmup > 0:
        g.scf(dd, ad, warmup)
    torch.cuda.synchronize()
    g.profile(True)
    t0 = time.perf_counter()
    it, res, _ = g.scf(dd, ad, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sweep_ms, launches = g.profile_read()
    g.profile(False)
    info = dict(g.info)
    g.close()
    return dt, it, sweep_ms, launches, info, res


def cpu_baseline(sp, d0, a0, n_angles):
    """The oracle as it stands, timed on a bounded sample: the complete
    sweep (node values, start values, both marches, pole sums) of the first
    n_angles Fermi-surface angles of the same workload."""
    from oracle import sweep as osw
    sys.path.insert(0, os.path.join(HERE, "tests"))
    from helpers import oracle_grain
    og = oracle_grain(sp)
    eps = 1j * og.zp * og.tt
    steps = 0
    t0 = time.perf_counter()
    for k in range(n_angles):
        data = og.data(k)
        dn, an = og.node_values(k, data, d0, a0)
        g0, gt0 = og.start_values(k, data, dn, an, eps, None)
        gn, gtn, _, _ = osw.march(data, dn, an, eps, og.q, g0, gt0)
        osw.node_sums(gn, gtn, dn, og.rp, og.tt)
        steps += 2 * og.n_poles * int(np.sum(og.tables[k].nnodes + 1))
    dt = time.perf_counter() - t0
    return steps / dt, dt, steps


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2205_15000_amd as qs
    from paper_2205_15000_amd import workloads as wl

    sp = wl.spec(WORKLOAD)
    d0 = wl.initial_delta(WORKLOAD, sp)
    a0 = wl.initial_A(WORKLOAD, sp)
    print("bench: %s mixed, %d warmup + %d timed iterations" % (WORKLOAD, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    dt, it, sweep_ms, launches, info, res = timed_scf(qs, torch, sp, "mixed", d0, a0, args.steps, args.warmup)
    steps_iter = info["steps_per_sweep"]
    value = steps_iter * it / dt
    ms_step = 1e3 * dt / it
    flops_launch = FLOPS_PER_STEP * steps_iter + FLOPS_PER_NODE_POLE * info["n_nodes"] * sp["n_poles"]
    avg_ms = sweep_ms / max(launches, 1)
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": it,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "d-wave [110] square 40 xi0, 400x400, 64 angles, 64 poles, t=0.1, "
                               "1 flux quantum, kappa=20, 1 vortex (Picard iterations)",
                   "name": WORKLOAD, "precision": "fp32 sweep / fp64 sums",
                   "steps_per_iteration": steps_iter, "segments": info["n_segments"],
                   "nodes": info["n_nodes"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_VALU_TFLOPS, "traffic": SWEEP_TRAFFIC_BYTES,
                     "kernel": "sweep_kernel<float,2,0>", "avg_launch_ms": avg_ms,
                     "flops_per_launch": flops_launch,
                     "peak_fp32_packed_published": PEAK_FP32_PACKED_TFLOPS},
        "sweep_only_steps_per_s": steps_iter / (avg_ms * 1e-3),
    }
    if not args.skip_fp64:
        print("bench: %s fp64" % WORKLOAD, file=sys.stderr, flush=True)
        dt64, it64, sms64, l64, _, _ = timed_scf(qs, torch, sp, "fp64", d0, a0, args.steps, args.warmup)
        v64 = steps_iter * it64 / dt64
        avg64 = sms64 / max(l64, 1)
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * dt64 / it64, "sweep_avg_launch_ms": avg64,
                       "sweep_only_steps_per_s": steps_iter / (avg64 * 1e-3),
                       "roofline_frac": flops_launch / (avg64 * 1e-3) / 1e12 / PEAK_VALU_TFLOPS}
        out["mixed_over_fp64"] = value / v64
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline (%d angles)" % args.cpu_angles, file=sys.stderr, flush=True)
        v, t, st = cpu_baseline(sp, d0, a0, args.cpu_angles)
        out["cpu_baseline"] = {"value": v, "unit": "trajectory-steps/s", "cores": 1, "kind": "oracle",
                               "sample": "oracle sweep (interpolation, both marches, pole sums) of %d of the "
                                         "64 angles of the same workload, first iteration: %d steps in %.1f s"
                                         % (args.cpu_angles, st, t)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
