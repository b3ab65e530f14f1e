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

Other measurements of the same library (one JSON line each; not the
headline):
    --mode accel [--iters N --tol T --accel-workload NAME]
                                  Picard against Polyak's heavy ball and BB: iterations
                                  to a global error below tol (default 1e-6, benchmark workload)
    --mode converge [--iters N]   mixed and FP64 Picard runs from the same
                                  start; difference of the final states
    --mode ldos [--prior N --bc-iters K]
                                  LDOS of the 512x512 [110] square, 256 angles,
                                  512 real energies, K boundary iterations
    --mode batch [--grains N --iters K]
                                  N seeded grains iterated together (persistent
                                  tile-queue sweep, hipGraph replay)
    --mode adjoint [--iters K]    FP64 sweep and its reverse mode on the 200x200
                                  d-wave disc (48 poles, 2 flux quanta)
    --mode lanes [--workload NAME]
                                  sweep time at every energies-per-lane setting,
                                  both precisions (default: the 48-pole disc)
    --mode valu                   sustained FP32 fma / rsq / sqrt / rcp rates of
                                  the device (the issue ceiling of the sweep)
    --mode vortex                 the paper's demonstration (s-wave disc, vortex,
                                  600x600): iterations of Picard, Polyak, BB and
                                  CongAcc to 1e-5, then the LDOS post-process
                                  (720 angles, 128 energies, to 1e-4)
    --mode errors                 mixed against FP64 per result on the 400x400
                                  workload: Delta, j, Omega, A, <g>, LDOS, and
                                  the self-consistent Delta (CongAcc to 1e-8,
                                  up to one global phase)
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
# Algorithmic work per trajectory step: the method's nominal count, about 59
# flops for the implicit-midpoint update (App. C, two square roots and two
# divisions included) plus the Green's functions and pole sums of a node
# (about 75 flops per node and pole, i.e. about 37 per step): 96 flops.
FLOPS_PER_STEP = 96
# A recount of the final formulas (complex ops expanded, sqrt and reciprocal
# one flop each; the step solved for its midpoint value): 47 per step plus
# 82 per (node, pole); reported beside.
RECOUNT_PER_STEP = 47
RECOUNT_PER_NODE_POLE = 82
PEAK_FP32_TFLOPS = 157.3     # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6      # MI355X published FP64 vector peak
# unpacked FP32 issues at the FP64 rate: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
UNPACKED_FP32_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# HBM bytes per sweep launch (mixed) from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs scaled by a plain-copy calibration (profiles/sweep_kernel_d110_square_400.md);
# None whenever the kernel changed after the counters were taken.
SWEEP_TRAFFIC_BYTES = 5.737e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-angles", type=int, default=4)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--mode", choices=["iteration", "converge", "accel", "ldos", "batch", "adjoint", "lanes", "valu",
                                       "vortex", "errors"],
                    default="iteration")
    ap.add_argument("--workload", default="d_disc_200")
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--prior", type=int, default=4000)
    ap.add_argument("--bc-iters", type=int, default=20)
    ap.add_argument("--grains", type=int, default=64)
    ap.add_argument("--accel-workload", default=WORKLOAD)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--ldos-angles", type=int, default=720)
    return ap.parse_args()


def timed_scf(qs, torch, sp, precision, d0, a0, steps, warmup):
    """warmup + steps Picard iterations from (d0, a0); only the last steps
    are timed.  Also returns the final state and, from one more sweep
    outside the timed region, its current and free energy."""
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
    info["energies_per_lane"], info["lanes_per_segment"] = g.lanes()
    info["pairing"], info["swept_steps_per_sweep"] = g.pairing()[1:]
    info["wide_segments"] = g.split()[1]
    _, j, om = g.sweep(dd, ad)
    final = {"delta": dd.cpu().numpy(), "A": ad.cpu().numpy(), "j": j.cpu().numpy(), "omega": om}
    g.close()
    return dt, it, sweep_ms, launches, info, res, final


def error_vs_fp64(mixed, fp64, mask, delta0):
    """Mixed against FP64 after the same iterations from the same start:
    the largest |Delta| difference on grain cells in units of Delta0 and the
    relative differences of j, A and the free energy."""
    dm, df = mixed["delta"][:, mask], fp64["delta"][:, mask]

    def rel(a, b):
        n = np.linalg.norm(b.ravel())
        return float(np.linalg.norm((a - b).ravel()) / n) if n > 0 else float(np.linalg.norm(a.ravel()))
    return {"delta_max_abs_over_delta0": float(np.max(np.abs(dm - df)) / delta0),
            "j_rel_l2": rel(mixed["j"], fp64["j"]), "A_rel_l2": rel(mixed["A"], fp64["A"]),
            "omega_rel": float(abs(mixed["omega"] - fp64["omega"]) / abs(fp64["omega"])),
            "tolerance_delta_over_delta0": 1e-4}


_CPU = {}


def _oracle_angles(ks):
    """The oracle's complete sweep (node values, start values, both marches,
    pole sums) of the angles ks; returns the trajectory steps done."""
    from oracle import sweep as osw
    og, d0, a0 = _CPU["og"], _CPU["d0"], _CPU["a0"]
    eps = 1j * og.zp * og.tt
    steps = 0
    for k in ks:
        data = og.data(k)
        dn, an = og.node_values(k, data, d0, a0)
        g0, gt0 = og.start_values(k, data, dn, an, eps, None)
        gn, gtn, _, _ = osw.march(data, dn, an, eps, og.q, g0, gt0)
        osw.node_sums(gn, gtn, dn, og.rp, og.tt)
        steps += 2 * og.n_poles * int(np.sum(og.tables[k].nnodes + 1))
    return steps


def cpu_baseline(sp, d0, a0, n_angles, workers):
    """The oracle as it stands on the host cores, before any GPU use: the
    first iteration's sweep of n_angles angles on one core, then of every
    angle with the angles split over `workers` forked processes."""
    sys.path.insert(0, os.path.join(HERE, "tests"))
    from helpers import oracle_grain
    _CPU.update(og=oracle_grain(sp), d0=d0, a0=a0)
    t0 = time.perf_counter()
    st1 = _oracle_angles(range(n_angles))
    dt1 = time.perf_counter() - t0
    out = {"one_core": (st1 / dt1, dt1, st1)}
    if workers > 1:
        import multiprocessing as mp
        nth = sp["n_theta"]
        chunks = [list(range(w, nth, workers)) for w in range(workers)]
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(workers) as pool:
            stw = sum(pool.map(_oracle_angles, chunks))
        dtw = time.perf_counter() - t0
        out["all_cores"] = (stw / dtw, dtw, stw)
    return out


def host_cores():
    """Cores this process may run on, capped at the 16 a one-GPU share holds."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _load_workloads():
    """workloads.py by path: importing the package would load the library,
    and the CPU baseline runs before anything touches the GPU."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_qc_workloads", os.path.join(HERE, "paper_2205_15000_amd", "workloads.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def mode_converge(qs, torch, wl, iters):
    """Mixed and FP64 Picard runs of the benchmark workload from the same
    start: residual histories and the difference of the final fields."""
    sp = wl.spec(WORKLOAD)
    d0 = wl.initial_delta(WORKLOAD, sp)
    a0 = wl.initial_A(WORKLOAD, sp)
    out, runs = {}, {}
    for prec in ("mixed", "fp64"):
        print("bench: converge %s, %d iterations" % (prec, iters), file=sys.stderr, flush=True)
        g = qs.Grain(sp, prec)
        dd = torch.as_tensor(d0).cuda()
        ad = torch.as_tensor(a0).cuda()
        t0 = time.perf_counter()
        it, res, conv = g.scf(dd, ad, iters, tol=1e-10)
        torch.cuda.synchronize()
        runs[prec] = {"iters": it, "s": time.perf_counter() - t0, "res_first": res[1, :4].tolist(),
                      "res_last": res[it - 1, :4].tolist()}
        out[prec] = (dd.cpu().numpy(), ad.cpu().numpy(), res[:it, :4])
        g.close()
    m = qs.Plan(dict(sp, n_theta=4)).mask()
    dm, df = out["mixed"][0][:, m], out["fp64"][0][:, m]
    hist = np.nanmax(np.abs(out["mixed"][2][1:] - out["fp64"][2][1:]) / np.abs(out["fp64"][2][1:]))
    return {"metric": "mixed vs FP64 final state after Picard iterations", "workload": WORKLOAD,
            "iterations": iters, "runs": runs,
            "max_abs_delta_diff_over_delta0": float(np.max(np.abs(dm - df)) / wl.DELTA0),
            "rel_l2_delta_diff": float(np.linalg.norm(dm - df) / np.linalg.norm(df)),
            "A_max_abs_diff": float(np.max(np.abs(out["mixed"][1] - out["fp64"][1]))),
            "A_max": float(np.max(np.abs(out["fp64"][1]))),
            "residual_history_max_rel_diff": float(hist)}


def mode_accel(qs, torch, wl, iters, tol, name=WORKLOAD):
    """Picard (step 1) against Polyak's heavy ball (step 2, drag 0.5),
    Barzilai-Borwein (first step 1) and CongAcc (first step 0.5), the
    defaults App. E lists, on the benchmark workload, mixed, from the same
    start: iterations and time until every global error is below tol."""
    sp = wl.spec(name)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    runs = {}
    for kind, alpha in (("picard", 1.0), ("polyak", 2.0), ("bb", 1.0), ("congacc", 0.5)):
        print("bench: accel %s, up to %d iterations" % (kind, iters), file=sys.stderr, flush=True)
        g = qs.Grain(sp, "mixed")
        g.set_accelerator(kind, 0.5)
        dd = torch.as_tensor(d0).cuda()
        ad = torch.as_tensor(a0).cuda()
        t0 = time.perf_counter()
        try:
            it, res, conv = g.scf(dd, ad, iters, tol=tol, alpha=alpha)
            torch.cuda.synchronize()
            runs[kind] = {"step": alpha, "iters": it, "converged": bool(conv), "s": time.perf_counter() - t0,
                          "res_last": res[it - 1, :4].tolist()}
        except qs.QcError as e:
            runs[kind] = {"step": alpha, "diverged": str(e)}
        g.close()
    return {"metric": "iterations to a global error below tol, Picard vs Polyak vs BB vs CongAcc (mixed)", "workload": name,
            "tol": tol, "max_iters": iters, "drag": 0.5, "runs": runs}


def mode_ldos(qs, torch, wl, n_prior, bc_iters):
    """LDOS of the 512x512 [110] square: an FP64 prior solve at 64 angles
    (CongAcc, to a global error of 1e-6 or n_prior iterations), then 256
    angles x 512 real energies with bc_iters boundary iterations (Delta and
    A frozen)."""
    name = "d110_square_512_ldos"
    sp = wl.spec(name)
    d0 = torch.as_tensor(wl.initial_delta(name, sp)).cuda()
    a0 = torch.as_tensor(wl.initial_A(name, sp)).cuda()
    print("bench: ldos prior solve, up to %d iterations" % n_prior, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    g = qs.Grain(dict(sp, n_theta=64), "fp64")
    g.set_accelerator("congacc")
    prior_it, prior_res, prior_conv = g.scf(d0, a0, n_prior, tol=1e-6, alpha=0.5)
    torch.cuda.synchronize()
    g.close()
    prior_s = time.perf_counter() - t0
    en = wl.ldos_energies(512)
    gl = qs.Grain(sp, "mixed")
    gl.profile(True)
    print("bench: ldos, %d energies, %d boundary iterations" % (len(en), bc_iters), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    o = gl.ldos(d0, a0, en, 0.01 * wl.DELTA0, bc_iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, nl = gl.profile_read()
    steps = gl.info["steps_per_sweep"] // sp["n_poles"] * len(en) * (bc_iters + 1)
    # with angle pairs and the symmetric energy set the boundary iterations
    # march the lower angle of each pair, and so does the output pass when
    # the pairs share their rotate-back corners
    paired = bool(gl.pairing()[1]) and bool(np.allclose(np.sort(en), -np.sort(en)[::-1], rtol=0, atol=1e-12))
    out_paired = paired and gl.rotate_fold()
    per_iter = gl.info["steps_per_sweep"] // sp["n_poles"] * len(en)
    marched = (per_iter // 2 if paired else per_iter) * bc_iters + (per_iter // 2 if out_paired else per_iter)
    o = o.cpu().numpy()
    gl.close()
    return {"metric": "LDOS trajectory-steps/s", "workload": name, "energies": len(en), "bc_iters": bc_iters,
            "value": steps / dt, "unit": "trajectory-steps/s", "seconds": dt, "steps": steps,
            "boundary_iterations_paired": paired, "output_pass_paired": out_paired, "marched_steps": marched, "marched_steps_per_s": marched / dt,
            "sweep_kernel_ms": ms, "sweep_launches": nl, "sweep_only_steps_per_s": steps / (ms * 1e-3),
            "prior_solve_s": prior_s, "prior_iters": prior_it, "prior_converged": bool(prior_conv),
            "prior_res_last": prior_res[prior_it - 1, :4].tolist(), "finite": bool(np.isfinite(o).all())}


def mode_batch(qs, torch, wl, n, iters):
    """n seeded grains (64x64 to 512x512, 32-128 angles, 32-128 poles)
    iterated together in the mixed path: eager and hipGraph timings after
    the autotuner has picked the energies per lane."""
    specs = wl.batch_specs(n)
    t0 = time.perf_counter()
    grains = []
    for i, sp in enumerate(specs):
        grains.append(qs.Grain(sp, "mixed"))
        if i % 8 == 7:
            print("bench: created %d grains" % (i + 1), file=sys.stderr, flush=True)
    b = qs.Batch(grains)
    for i, sp in enumerate(specs):
        b.set_fields(i, torch.as_tensor(wl.batch_initial_delta(sp, i)).cuda(),
                     torch.zeros((2, sp["ny"], sp["nx"]), dtype=torch.float64).cuda())
    setup_s = time.perf_counter() - t0
    info = b.info()
    b.iterate(1, graph=False)
    epl = b.autotune(1)
    print("bench: batch autotuned to %d energies per lane" % epl, file=sys.stderr, flush=True)
    ms_e = b.iterate(2, graph=False)
    b.iterate(iters, graph=True)  # captures the graphs
    ms_g = b.iterate(iters, graph=True)
    d, _ = b.get_fields(0)
    st = info["steps_per_iteration"]
    return {"metric": "batched trajectory-steps/s", "grains": n, "unit": "trajectory-steps/s",
            "value": st * iters / (ms_g * 1e-3), "graph_ms_per_iteration": ms_g / iters,
            "eager_ms_per_iteration": ms_e / 2, "eager_steps_per_s": st * 2 / (ms_e * 1e-3),
            "steps_per_iteration": st, "energies_per_lane": epl, "tiles": info["tiles"], "setup_s": setup_s,
            "finite": bool(torch.isfinite(d).all())}


def mode_adjoint(qs, torch, wl, iters):
    """Forward sweep and reverse mode (frozen boundary store) of the FP64
    d-wave disc, R = 20 xi0 on 200x200, 64 angles, 48 poles: wall time per
    call with inputs resident, after one warmup each; the reverse mode with
    checkpoints every 32 steps (the default) and with everything stored."""
    name = "d_disc_200"
    sp = wl.spec(name)
    g = qs.Grain(sp, "fp64")
    dd = torch.as_tensor(wl.initial_delta(name, sp)).cuda()
    ad = torch.as_tensor(wl.initial_A(name, sp)).cuda()
    rng = np.random.default_rng(5)
    gdn = torch.as_tensor(rng.standard_normal(dd.shape) + 1j * rng.standard_normal(dd.shape)).cuda()
    gj = torch.as_tensor(rng.standard_normal((2, sp["ny"], sp["nx"]))).cuda()
    g.sweep(dd, ad)
    g.sweep(dd, ad)
    g.sweep_adjoint(dd, ad, gdn, gj, 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        g.sweep(dd, ad, total=False)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / iters
    # the default: checkpoints every 32 steps
    t0 = time.perf_counter()
    for _ in range(iters):
        gd, ga = g.sweep_adjoint(dd, ad, gdn, gj, 1.0)
    torch.cuda.synchronize()
    adj = (time.perf_counter() - t0) / iters
    # gamma~ and its adjoint terms stored at every node
    g.set_adjoint_checkpoint(0)
    g.sweep_adjoint(dd, ad, gdn, gj, 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        gds, gas = g.sweep_adjoint(dd, ad, gdn, gj, 1.0)
    torch.cuda.synchronize()
    adjs = (time.perf_counter() - t0) / iters
    same = float(max((gds - gd).abs().max() / gd.abs().max(), (gas - ga).abs().max() / ga.abs().max()))
    steps = g.steps_per_sweep
    finite = bool(torch.isfinite(torch.view_as_real(gd)).all() and torch.isfinite(ga).all())
    g.close()
    return {"metric": "adjoint sweep time", "workload": name, "precision": "fp64", "iterations": iters,
            "forward_ms": 1e3 * fwd, "adjoint_ms": 1e3 * adj, "adjoint_over_forward": adj / fwd,
            "checkpoint_every": 32, "adjoint_stored_ms": 1e3 * adjs, "stored_vs_checkpointed_max_rel_diff": same,
            "forward_steps": steps, "forward_steps_per_s": steps / fwd, "finite": finite}


def mode_lanes(qs, torch, wl, name, iters):
    """Average sweep-kernel time (HIP events) at each energies-per-lane
    setting and at the automatic choice, mixed and FP64, same inputs."""
    sp = wl.spec(name)
    d0 = torch.as_tensor(wl.initial_delta(name, sp)).cuda()
    a0 = torch.as_tensor(wl.initial_A(name, sp)).cuda()
    rows = []
    for prec in ("mixed", "fp64"):
        g = qs.Grain(sp, prec)
        g.sweep(d0, a0)  # warm-up of the grain's buffers and clocks
        for epl in (1, 2, 3, 4, 8, 0):
            g.set_lanes(epl)
            g.reset_bc()
            g.sweep(d0, a0)
            g.sweep(d0, a0)
            torch.cuda.synchronize()
            g.profile(True)
            for _ in range(iters):
                g.sweep(d0, a0, total=False)
            torch.cuda.synchronize()
            ms, n = g.profile_read()
            g.profile(False)
            e, G = g.lanes()
            rows.append({"precision": prec, "requested": epl, "energies_per_lane": e, "lanes_per_segment": G,
                         "sweep_ms": ms / max(n, 1)})
        # the split launch shape at the automatic lane shape (0: off)
        g.set_lanes(0)
        for frac in (0.0, 0.5, 0.6, 0.7, 0.75, 0.8, 0.85, 0.9, 0.95):
            g.set_split(frac)
            g.reset_bc()
            g.sweep(d0, a0)
            g.sweep(d0, a0)
            torch.cuda.synchronize()
            g.profile(True)
            for _ in range(iters):
                g.sweep(d0, a0, total=False)
            torch.cuda.synchronize()
            ms, n = g.profile_read()
            g.profile(False)
            rows.append({"precision": prec, "split": frac, "wide_segments": g.split()[1], "sweep_ms": ms / max(n, 1)})
        g.close()
    return {"metric": "sweep time per lane shape", "workload": name, "n_poles": sp["n_poles"], "rows": rows}


def mode_valu(qs):
    """Sustained rate of single FP32 VALU operations with every CU busy:
    the issue ceiling the sweep kernels run against (a wave64 instruction
    issues 16 lanes per cycle per SIMD, 1024 SIMDs)."""
    r = {op: qs.valu_rate(op) for op in ("fma", "rsq", "sqrt", "rcp")}
    return {"metric": "sustained FP32 VALU rate", "unit": "lane ops/s",
            "fma": r["fma"], "rsq": r["rsq"], "sqrt": r["sqrt"], "rcp": r["rcp"],
            "fma_tflops": 2 * r["fma"] / 1e12, "fma_over_published_78_6": 2 * r["fma"] / 1e12 / PEAK_VALU_TFLOPS,
            "implied_clock_ghz": r["fma"] / (1024 * 16) / 1e9,
            "transcendental_over_fma": {op: r[op] / r["fma"] for op in ("rsq", "sqrt", "rcp")}}


def mode_vortex(qs, torch, wl, max_iter, ldos_angles):
    """The demonstration of Sec. IV (App. B listing): every accelerator of
    App. E from the same start, FP64, to the listing's tolerance 1e-5; then
    the LDOS post-process of the converged CongAcc state (Sec. IV listing:
    energies 0..0.5, broadening 0.008, iterated to 1e-4) in the mixed path,
    and the save / restore round trip of the state."""
    name = "swave_disc_vortex"
    sp = wl.spec(name)
    d0 = torch.as_tensor(wl.initial_delta(name, sp)).cuda()
    a0 = torch.as_tensor(wl.initial_A(name, sp)).cuda()
    paper = {"picard": "F", "polyak": "F", "bb": 45, "congacc": 42}
    runs = {}
    keep = None
    for kind, alpha in (("picard", 1.0), ("polyak", 2.0), ("bb", 1.0), ("congacc", 0.5)):
        print("bench: vortex %s" % kind, file=sys.stderr, flush=True)
        g = qs.Grain(sp, "fp64")
        g.set_accelerator(kind, 0.5)
        d, a = d0.clone(), a0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            it, res, conv = g.scf(d, a, max_iter, tol=1e-5, alpha=alpha)
            torch.cuda.synchronize()
            runs[kind] = {"step": alpha, "iters": it, "converged": bool(conv), "s": time.perf_counter() - t0,
                          "res_last": res[it - 1, :4].tolist(), "paper_iters": paper[kind]}
        except qs.QcError as e:
            runs[kind] = {"step": alpha, "diverged": str(e), "paper_iters": paper[kind]}
        if kind == "congacc":
            t0 = time.perf_counter()
            st = g.get_state().clone()
            g2 = qs.Grain(sp, "fp64")
            g2.set_state(st)
            dn, _, _ = g2.sweep(d, a)
            torch.cuda.synchronize()
            runs[kind]["resume_s"] = time.perf_counter() - t0
            runs[kind]["resume_first_map_max_change_over_delta0"] = float((dn - d).abs().max()) / wl.DELTA0
            g2.close()
            keep = (d, a)
        g.close()
    d, a = keep
    print("bench: vortex LDOS, %d angles" % ldos_angles, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    gl = qs.Grain(dict(sp, n_theta=ldos_angles), "mixed")
    setup = time.perf_counter() - t0
    en = wl.vortex_ldos_energies(128)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ld, iters = gl.ldos_converge(d, a, en, 0.008, 1e-4, 1000, energies_per_block=32)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps_bc = gl.info["steps_per_sweep"] // sp["n_poles"] * len(en)
    ld = ld.cpu().numpy()
    X, Y = wl.centres(sp)
    r = np.hypot(X, Y)
    gl.close()
    return {"metric": "iterations to 1e-5 per accelerator, and the LDOS post-process", "workload": name,
            "precision_scf": "fp64", "runs": runs,
            "ldos": {"angles": ldos_angles, "energies": len(en), "broadening": 0.008, "tol": 1e-4,
                     "sweeps_slowest_block": iters, "seconds": dt, "plan_and_upload_s": setup,
                     "steps_per_sweep_all_energies": steps_bc,
                     "core_N0": float(ld[0][r < 0.3].mean()), "ring_8_9_N0": float(ld[0][(r > 8) & (r < 9)].mean()),
                     "finite": bool(np.isfinite(ld).all())}}


def mode_errors(qs, torch, wl, scf_iters):
    """Mixed against FP64 per result on the 400x400 [110] workload: the
    first three chained maps against the oracle's stored values (Delta, j,
    Omega), the A-solve of each precision's current, the Green's function
    average and the LDOS (64 angles, 16 energies) against the FP64 path,
    and the self-consistent Delta: FP64 CongAcc to 1e-8, then the mixed path
    from that state to 1e-8, compared up to one global phase (a common phase
    factor leaves the gap equation and the current unchanged)."""
    name = WORKLOAD
    sp = wl.spec(name)
    gold = np.load(os.path.join(HERE, "tests", "golden", name + "_iter3.npz"))
    cells = gold["cells"]
    d0 = torch.as_tensor(wl.initial_delta(name, sp)).cuda()
    a0 = torch.as_tensor(wl.initial_A(name, sp)).cuda()
    out = {"metric": "mixed vs FP64 error per result", "workload": name, "delta0": wl.DELTA0}
    maps = {}
    for prec in ("mixed", "fp64"):
        print("bench: errors, three maps %s" % prec, file=sys.stderr, flush=True)
        g = qs.Grain(sp, prec)
        d, a = d0.clone(), a0.clone()
        rows = []
        for i in range(3):
            dn, j, om = g.sweep(d, a)
            A, _ = g.solve_A(j, B=False)
            dg = dn.cpu().numpy().reshape(1, -1)[:, cells]
            jg = j.cpu().numpy().reshape(2, -1)[:, cells]
            rows.append({"delta_max_abs_over_delta0": float(np.max(np.abs(dg - gold["delta_new"][i])) / wl.DELTA0),
                         "j_max_abs_over_max_j": float(np.max(np.abs(jg - gold["j"][i])) / np.max(np.abs(gold["j"][i]))),
                         "omega_rel": float(abs(om - gold["omega_total"][i]) / abs(gold["omega_total"][i]))})
            maps.setdefault(prec, []).append(A.cpu().numpy())
            d, a = dn, A
        out["maps_vs_oracle_" + prec] = rows
        g.close()
    out["A_max_abs_over_max_A"] = [float(np.max(np.abs(x - y)) / np.max(np.abs(y)))
                                   for x, y in zip(maps["mixed"], maps["fp64"])]
    res = {}
    for prec in ("mixed", "fp64"):
        print("bench: errors, <g> and LDOS %s" % prec, file=sys.stderr, flush=True)
        g = qs.Grain(sp, prec)
        g.sweep(d0, a0)
        gav = g.green_average(d0, a0).cpu().numpy()
        ld = g.ldos(d0, a0, np.linspace(-1.5, 1.5, 16) * wl.DELTA0, 0.01 * wl.DELTA0, 10).cpu().numpy()
        res[prec] = (gav, ld)
        g.close()
    out["green_average_max_abs_over_max"] = float(np.max(np.abs(res["mixed"][0] - res["fp64"][0]))
                                                  / np.max(np.abs(res["fp64"][0])))
    out["ldos_max_abs"] = float(np.max(np.abs(res["mixed"][1] - res["fp64"][1])))
    out["ldos_max"] = float(np.max(np.abs(res["fp64"][1])))
    # the self-consistent state: FP64 with CongAcc to 1e-8 from the start,
    # then the mixed path from that state to 1e-8 (its own fixed point next
    # to the FP64 one); independent runs from the start can settle in
    # different states (vortex positions are not unique)
    sc = {}
    d, a = d0.clone(), a0.clone()
    for prec in ("fp64", "mixed"):
        print("bench: errors, CongAcc to 1e-8 %s" % prec, file=sys.stderr, flush=True)
        g = qs.Grain(sp, prec)
        g.set_accelerator("congacc")
        t0 = time.perf_counter()
        it, hist, conv = g.scf(d, a, scf_iters, tol=1e-8, alpha=0.5)
        torch.cuda.synchronize()
        sc[prec] = {"iters": it, "converged": bool(conv), "s": time.perf_counter() - t0,
                    "res_last": hist[it - 1, :4].tolist(), "delta": d.cpu().numpy().copy()}
        g.close()
    m = qs.Plan(dict(sp, n_theta=4)).mask()
    x, y = sc["fp64"]["delta"][:, m], sc["mixed"]["delta"][:, m]
    chi = float(np.angle(np.vdot(x, y)))
    raw = np.max(np.abs(y - x)) / wl.DELTA0
    diff = np.max(np.abs(y * np.exp(-1j * chi) - x)) / wl.DELTA0
    for prec in sc:
        sc[prec].pop("delta")
    out["self_consistent"] = {"runs": sc, "mixed_started_from": "the FP64 self-consistent state",
                              "global_phase_rad": chi,
                              "delta_max_abs_over_delta0_raw": float(raw),
                              "delta_max_abs_over_delta0": float(diff), "tolerance": 1e-4}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path, so --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    cpu = None
    if args.mode == "iteration" and not args.no_cpu_baseline:
        # on the host cores, before anything touches the GPU (the pool forks)
        wl0 = _load_workloads()
        sp0 = wl0.spec(WORKLOAD)
        workers = host_cores()
        print("bench: oracle CPU baseline (%d angles on one core, all angles on %d processes)"
              % (args.cpu_angles, workers), file=sys.stderr, flush=True)
        cpu = cpu_baseline(sp0, wl0.initial_delta(WORKLOAD, sp0), wl0.initial_A(WORKLOAD, sp0),
                           args.cpu_angles, workers)
        cpu["workers"] = workers

    import torch
    import paper_2205_15000_amd as qs
    from paper_2205_15000_amd import workloads as wl

    if args.mode != "iteration":
        if args.mode == "converge":
            res = mode_converge(qs, torch, wl, args.iters or 3000)
        elif args.mode == "accel":
            res = mode_accel(qs, torch, wl, args.iters or 3000, args.tol, args.accel_workload)
        elif args.mode == "ldos":
            res = mode_ldos(qs, torch, wl, args.prior, args.bc_iters)
        elif args.mode == "adjoint":
            res = mode_adjoint(qs, torch, wl, args.iters or 5)
        elif args.mode == "lanes":
            res = mode_lanes(qs, torch, wl, args.workload, args.iters or 8)
        elif args.mode == "valu":
            res = mode_valu(qs)
        elif args.mode == "vortex":
            res = mode_vortex(qs, torch, wl, args.iters or 1000, args.ldos_angles)
        elif args.mode == "errors":
            res = mode_errors(qs, torch, wl, args.iters or 9000)
        else:
            res = mode_batch(qs, torch, wl, args.grains, args.iters or 6)
        print(json.dumps(res), flush=True)
        return

    sp = wl.spec(WORKLOAD)
    d0 = wl.initial_delta(WORKLOAD, sp)
    a0 = wl.initial_A(WORKLOAD, sp)
    print("bench: %s mixed, %d warmup + %d timed iterations" % (WORKLOAD, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    dt, it, sweep_ms, launches, info, res, fin_m = timed_scf(qs, torch, sp, "mixed", d0, a0, args.steps,
                                                             args.warmup)
    steps_iter = info["steps_per_sweep"]
    # with angle pairs the sweep marches half of the workload's steps (the
    # other half follows exactly from the symmetry); the roofline counts the
    # marched work
    swept = info["swept_steps_per_sweep"]
    value = steps_iter * it / dt
    ms_step = 1e3 * dt / it
    flops_launch = FLOPS_PER_STEP * swept
    recount = (RECOUNT_PER_STEP * swept
               + RECOUNT_PER_NODE_POLE * info["n_nodes"] * sp["n_poles"] * swept / steps_iter)
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
                   "name": WORKLOAD, "precision": "fp32 sweeps / fp64 pole, angle and cell sums",
                   "steps_per_iteration": steps_iter, "marched_steps_per_iteration": swept,
                   "angle_pairs": bool(info["pairing"]), "segments": info["n_segments"],
                   "nodes": info["n_nodes"], "wide_segments": info["wide_segments"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": SWEEP_TRAFFIC_BYTES,
                     "kernel": "sweep_kernel<float,%d,0>" % info["energies_per_lane"],
                     "flops_per_step": FLOPS_PER_STEP, "flops_per_launch": flops_launch,
                     "lanes_per_segment": info["lanes_per_segment"], "avg_launch_ms": avg_ms,
                     "unpacked_fp32_ceiling": UNPACKED_FP32_TFLOPS,
                     "frac_of_unpacked_fp32": achieved / UNPACKED_FP32_TFLOPS,
                     "recount_flops_per_launch": recount,
                     "recount_tflops": recount / (avg_ms * 1e-3) / 1e12},
        "sweep_only_steps_per_s": steps_iter / (avg_ms * 1e-3),
        "marched_steps_per_s": swept * it / dt,
    }
    # the ceiling the device sustains under a full VALU load (same run, same
    # device): FP32 fma rate with every CU busy
    fma = qs.valu_rate("fma")
    out["roofline"]["sustained_fma_tflops"] = 2 * fma / 1e12
    out["roofline"]["frac_of_sustained"] = achieved / (2 * fma / 1e12)
    if not args.skip_fp64:
        print("bench: %s fp64" % WORKLOAD, file=sys.stderr, flush=True)
        dt64, it64, sms64, l64, _, _, fin_d = timed_scf(qs, torch, sp, "fp64", d0, a0, args.steps, args.warmup)
        v64 = steps_iter * it64 / dt64
        avg64 = sms64 / max(l64, 1)
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * dt64 / it64, "sweep_avg_launch_ms": avg64,
                       "marched_steps_per_s": swept * it64 / dt64,
                       "sweep_only_steps_per_s": steps_iter / (avg64 * 1e-3),
                       "roofline_achieved": flops_launch / (avg64 * 1e-3) / 1e12, "roofline_peak": PEAK_FP64_TFLOPS,
                       "roofline_frac": flops_launch / (avg64 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
        out["mixed_over_fp64"] = value / v64
        mask = qs.Plan(dict(sp, n_theta=4)).mask()
        out["error_vs_fp64"] = error_vs_fp64(fin_m, fin_d, mask, wl.DELTA0)
        out["error_vs_fp64"]["iterations"] = args.warmup + args.steps
    if cpu is not None:
        v1, t1, s1 = cpu["one_core"]
        cb = {"value": v1, "unit": "trajectory-steps/s", "cores": 1, "kind": "oracle",
              "sample": "oracle sweep (interpolation, both marches, pole sums) of %d of the 64 angles of the "
                        "same workload, first iteration, one core: %d steps in %.1f s" % (args.cpu_angles, s1, t1),
              "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        if "all_cores" in cpu:
            vw, tw, sw = cpu["all_cores"]
            cb.update(value=vw, cores=cpu["workers"], one_core_value=v1,
                      sample="oracle sweep of all 64 angles of the same workload, first iteration, angles split "
                             "over %d processes: %d steps in %.1f s (one core, %d angles: %.3g steps/s)"
                             % (cpu["workers"], sw, tw, args.cpu_angles, v1))
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
