"""Benchmark of the FC-SDNN per-stage hot path on one MI355X.

Workload: the Mach-3 step channel ([0, 3] x [0, 1] with a step over
[0.6, 3] x [0, 0.2]; 22 overlapping subpatches of up to 112 x 109 points on a
h = 1/250 lattice, with one L-shaped C1 corner patch and one C2 corner patch;
inflow rho = 1.4, p = 1, u = 3; slip walls; SDNN artificial viscosity with
a classifier trained on the GPU by the library's own kernels at set-up;
spectral filter; adaptive step at CFL 0.5).  One benchmark step is one
solver time step: viscosity (classification, smoothing, blend), filter,
step size and the five SSPRK stages (fluxes, grouped FC derivative
contractions, viscous terms, update, boundary conditions, fringe
interpolation), replayed as one captured hipGraph.

Prints one JSON line: point-stage updates/s of the plain FP64 form (the
configuration as stated) and, in ``mixed``, of the split-BF16 contraction
form with its error against the FP64 run at equal step counts; the roofline
of the dominant kernel (the grouped contraction, timed with HIP events on
the solver stream) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2.5e15}
# HBM bytes per stage-contraction launch on the step channel (FP64): the
# launches the roofline times (the last step's stage contraction, back to
# back), from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by the
# factors a 256 MiB copy gives in the same runs.  The work per launch follows
# the flow (viscous lines are skipped where mu vanishes), so a figure holds
# for its kernel after the same number of steps and warm-up steps, and for
# the kernels as they were when the counters were taken.
STAGE_TRAFFIC_FP64 = {
    # profiles/stage_contraction_fp64_traffic.md (fetched + written MB)
    ("k_gemm_fp<double, 8, 1, 4, 2>", 2000, 20): 52.25e6,  # 28.58 + 23.67
    ("k_gemm_fp<double, 16, 1, 4, 1>", 2000, 20): 52.08e6,  # 28.55 + 23.53
    ("k_gemm_fp<double, 16, 1, 3, 2>", 2000, 20): 52.91e6,  # 29.55 + 23.36
}
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the derivative-sweep and classifier measurements")
    ap.add_argument("--eager", action="store_true", help="launch kernels one by one instead of replaying step graphs "
                                                           "(for per-dispatch counter runs)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="finish with three plain 256 MiB device copies (byte-counter calibration)")
    ap.add_argument("--stage-variant", default=None,
                    help="pin the FP64 stage-contraction tile shape (a kernel name as reported in roofline.kernel) "
                         "instead of tuning it (for counter runs, whose dispatch serialization skews the tuner)")
    ap.add_argument("--no-tiled", action="store_true",
                    help="skip the tiled step channel at 1.17e7 points (FP64 and split-BF16, 500 steps)")
    ap.add_argument("--tiled-steps", type=int, default=500)
    ap.add_argument("--tiled-only", action="store_true",
                    help="run only the tiled step channel (for its kernel profile); prints its object alone")
    ap.add_argument("--cpu-steps", type=int, default=10)
    return ap.parse_args()


def train_classifier(F, W, torch, steps=300, batch=4096):
    """Seeded training of the smoothness classifier on the GPU: synthetic
    lines through the solver's FC filter (d = 2, C = 27), 16-point windows,
    class-weighted Adam with the library's training kernels."""
    lines, pos, amp = W.classifier_lines(3000, seed_salt=51)
    filt = F.lines_apply(torch.tensor(lines, device="cuda"), "filter", 2, 27)
    lab = W.window_labels(pos, amp, lines)
    n = lines.shape[1]
    start = np.clip(np.arange(n) - 8, 0, n - 16)
    idx = torch.tensor(start[:, None] + np.arange(16)[None, :], device="cuda")
    wins = filt[:, idx].reshape(-1, 16)
    lo = wins.min(dim=1, keepdim=True).values
    hi = wins.max(dim=1, keepdim=True).values
    am = wins.abs().max(dim=1, keepdim=True).values
    rng_ = hi - lo
    keep = (rng_ >= 1e-3 * torch.clamp(am, min=1.0)).squeeze(1)
    x = ((wins - lo) / torch.where(rng_ > 0, rng_, torch.ones_like(rng_)))[keep].float().contiguous()
    y = torch.tensor(lab.reshape(-1), device="cuda")[keep].int().contiguous()
    counts = torch.bincount(y, minlength=3).double()
    cw = (counts.sum() / (3.0 * torch.clamp(counts, min=1.0))).float()
    g = W.rng(4, 52)
    params = torch.tensor(W.sdnn_blob(W.sdnn_init(g)), device="cuda")
    tr = F.SdnnTrainer(params, batch=batch, lr=2e-3)
    for _ in range(steps):
        sel = torch.tensor(g.integers(0, y.numel(), batch), device="cuda")
        tr.step(x[sel].contiguous(), y[sel].contiguous(), cw)
    torch.cuda.synchronize()
    return params.cpu().numpy()


def sweep_bench(F, W, torch):
    """Grouped derivative contraction on its own: 2000 patches with sides
    drawn from 64..256, four fields, d/dq1 and d/dq2 (FC d = 5, C = 27) in one
    launch, each precision autotuned; rates against each precision's MFMA peak
    and against the FP32 peak (FP32-equivalent work)."""
    sizes, fields = W.deriv_sweep(2000)
    x = torch.tensor(np.concatenate([f.ravel() for f in fields]), device="cuda")
    d1, d2 = torch.empty_like(x), torch.empty_like(x)
    out = {"workload": "2000 patches, sides U{64..256}, 4 fields, d/dq1 and d/dq2, FC d=5 C=27, one launch",
           "points": int(sum(int(a) * int(b) for a, b in sizes))}
    for prec in ("fp64", "fp32", "bf16x3"):
        sw = F.DerivSweep(sizes, 4, prec, d=5, C=27)
        sw.autotune(x, d1, d2)
        sw.profile(1)
        for _ in range(10):
            sw.run(x, d1, d2)
        r = sw.profile(-1)
        rate = r["flops"] / (r["avg_ms"] * 1e-3)
        own = PEAK["fp32"] if prec == "bf16x3" else PEAK[prec]
        out[prec] = {"ms": r["avg_ms"], "tflops": rate / 1e12, "frac_of_fp32_peak": rate / PEAK["fp32"],
                     "frac_of_own_peak": rate / own if prec != "bf16x3" else None,
                     "algorithmic_GBps": r["bytes"] / (r["avg_ms"] * 1e-3) / 1e9}
        del sw
    return out


def classifier_bench(F, W, torch, weights):
    """Window classification throughput: 10^7 windows of FC-filtered
    synthetic lines (smooth Fourier sums with 0-2 jumps), trained SDNN on
    the matrix cores vs the modal-decay fallback."""
    lines, _, _ = W.classifier_lines(20000, seed_salt=61)
    filt = F.lines_apply(torch.tensor(lines, device="cuda"), "filter", 2, 27)
    n = lines.shape[1]
    start = np.clip(np.arange(n) - 8, 0, n - 16)
    idx = torch.tensor(start[:, None] + np.arange(16)[None, :], device="cuda")
    base = filt[:, idx].reshape(-1, 16)
    nwin = 10_000_000
    wins = base.repeat((nwin + base.shape[0] - 1) // base.shape[0], 1)[:nwin].contiguous()
    p = torch.tensor(weights, device="cuda")
    out = {"windows": nwin}
    for name, fn in (("sdnn", lambda: F.sdnn_infer(p, wins)), ("modal", lambda: F.modal_infer(wins))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        out[name] = {"ms": ms, "windows_per_s": nwin / (ms * 1e-3)}
    return out


def make_solver(F, W, torch, weights, precision, stream, use_graph=True, specs=None):
    specs = W.step_channel() if specs is None else specs
    prm = F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="sdnn", filter=True, use_graph=use_graph,
                         precision=precision, sdnn_weights=weights, autotune=True)
    with torch.cuda.stream(stream):
        S = F.Solver(specs, prm, stream=stream)
        w = W.uniform_state(specs, W.STEP_INFLOW)
        for p in range(len(specs)):
            S.set_state(p, w[p])
    return S, specs


def timed_run(S, torch, stream, steps, warmup, retune=True):
    # The first advance tunes the contraction tile on the initial state, where
    # no viscous line is active yet; the last warm-up step tunes it again on
    # the developed flow (and captures the step graphs anew).
    if warmup > 0 and retune:
        S.advance(5 * (warmup - 1), sync=True)
        S.retune()
        S.advance(5, sync=True)
    elif warmup > 0:
        S.advance(5 * warmup, sync=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.advance(5 * steps)
    stream.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.advance(0, sync=True)  # raises if the state became non-finite
    return el


def field_errors(ref_solver, solver, specs):
    """Per-field max and RMS difference over all active points, relative to
    the field's largest magnitude in the reference run."""
    errs = {}
    for name in ("rho", "mx", "my", "E"):
        sel = [specs[p].mask if specs[p].mask is not None else np.ones(specs[p].shape, bool)
               for p in range(len(specs))]
        ref = np.concatenate([ref_solver.field(p, name)[sel[p]] for p in range(len(specs))])
        got = np.concatenate([solver.field(p, name)[sel[p]] for p in range(len(specs))])
        d = got - ref
        scale = max(np.abs(ref).max(), 1e-300)
        errs[name] = {"max_rel": float(np.abs(d).max() / scale), "rms_rel": float(np.sqrt((d * d).mean()) / scale)}
    return errs


def contraction_profile(S, torch, nsteps=20, reps=50):
    """Duration of the stage contraction: (1) HIP events around each launch in
    nsteps replayed steps (event-record nodes in the graph; the interval also
    holds the dispatch latency those nodes add), then (2) the last of those
    steps' stage contraction alone, reps launches back to back between two
    HIP events on the solver stream: the kernel's own average duration."""
    S.profile(True)
    S.advance(5 * nsteps, sync=True)
    graph = S.profile_read()
    S.profile(False)
    alone = S.profile_stage(reps)
    return alone, graph


def tiled_channel_run(F, W, torch, weights, steps, warmup=5):
    """The step channel tiled by 235 subpatches of uneven sizes (sides drawn
    from 150-300; 1.17e7 points, C1 and C2 corner patches): FP64 and
    split-BF16 runs of the same steps from the uniform inflow state, their
    throughput and the per-field difference of the split-BF16 state from the
    FP64 one after the run."""
    specs = W.step_channel_tiled()
    npts = int(sum(s.npoints() for s in specs))
    out = {"workload": "Mach-3 step channel tiled by %d subpatches of sides 150-300 (seeded), %d points, "
                       "SDNN viscosity, filter, CFL 0.5, FC-Gram d=2 C=27" % (len(specs), npts),
           "points": npts, "subpatches": len(specs), "steps": steps, "warmup": warmup}
    from paper_2506_19370_amd import _lib as L
    solvers = {}
    for prec in ("fp64", "bf16x3"):
        stream = torch.cuda.Stream()
        t0 = time.perf_counter()
        S, _ = make_solver(F, W, torch, weights, prec, stream, specs=specs)
        setup = time.perf_counter() - t0
        el = timed_run(S, torch, stream, steps, warmup)
        out[prec] = {"value": npts * 5 * steps / el, "unit": "point-stage updates/s", "ms_per_step": el / steps * 1e3,
                     "stage_kernel": L.gemm_variant_name(prec, S.stats()["stage_variant"]),
                     "host_setup_s": setup}
        if prec == "fp64":
            # the last step's stage contraction alone (useful flops of the
            # lines that step needed), as for the roofline of the main run
            pr = S.profile_stage(20)
            ach = pr["flops"] / (pr["avg_ms"] * 1e-3)
            out[prec]["stage_contraction"] = {"avg_launch_ms": pr["avg_ms"], "flops_per_launch": pr["flops"],
                                              "achieved_tflops": ach / 1e12, "frac_of_fp64_peak": ach / PEAK["fp64"],
                                              "algorithmic_bytes_per_launch": pr["bytes"]}
        solvers[prec] = S
    out["bf16x3"]["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["bf16x3"]["ms_per_step"]
    out["bf16x3"]["error_vs_fp64_after_%d_steps" % (steps + warmup)] = field_errors(solvers["fp64"],
                                                                                     solvers["bf16x3"], specs)
    del solvers
    torch.cuda.synchronize()
    return out


def cpu_baseline(W, steps):
    from threadpoolctl import threadpool_limits
    from oracle import solver as osolver
    specs = W.step_channel()
    with threadpool_limits(limits=1):
        O = osolver.Solver(osolver.patches_from_specs(specs),
                           osolver.Params(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True))
        O.set_prim(W.uniform_state(specs, W.STEP_INFLOW))
        t0 = time.perf_counter()
        for _ in range(steps):
            O.step()
        el = time.perf_counter() - t0
    npts = int(sum(s.npoints() for s in specs))
    return {"value": npts * 5 * steps / el, "unit": "point-stage updates/s", "cores": 1, "kind": "oracle",
            "sample": f"step channel, first {steps} steps (modal-indicator viscosity, filter), "
                      f"{npts} points, FP64 NumPy, 1 thread, {el:.1f} s"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 (multi-GPU sharding is a design "
                                   "note, not an implemented path)"}))
        sys.exit(2)
    import torch
    import paper_2506_19370_amd as F
    import workloads as W

    weights = train_classifier(F, W, torch)
    if a.tiled_only:
        print(json.dumps({"tiled_channel": tiled_channel_run(F, W, torch, weights, a.tiled_steps)}))
        return
    stream = torch.cuda.Stream()
    S, specs = make_solver(F, W, torch, weights, "fp64", stream, use_graph=not a.eager)
    if a.stage_variant:
        S.set_stage_variant(a.stage_variant)
    npts = int(sum(s.npoints() for s in specs))
    el = timed_run(S, torch, stream, a.steps, a.warmup, retune=not a.stage_variant)
    value = npts * 5 * a.steps / el
    prof, gprof = contraction_profile(S, torch)
    kernel_ms = prof["avg_ms"]
    achieved = prof["flops"] / (kernel_ms * 1e-3)
    from paper_2506_19370_amd import _lib as L
    kernel = L.gemm_variant_name("fp64", S.stats()["stage_variant"])
    traffic = STAGE_TRAFFIC_FP64.get((kernel, a.steps, a.warmup))
    out = {
        "metric": "point-stage updates/s, plain FP64 vs mixed-precision batched form at stated error",
        "value": value, "unit": "point-stage updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Mach-3 step channel [0,3]x[0,1], step [0.6,3]x[0,0.2], 22 subpatches "
                               "(C1 L-shaped + C2 corner patches), %d points, SDNN viscosity (GPU-trained), "
                               "filter, CFL 0.5, FC-Gram d=2 C=27" % npts,
                   "points": npts, "stages_per_step": 5},
        "roofline": {"bound": "mfma", "kernel": kernel + " (grouped FC stage contraction, autotuned tile)",
                     "achieved": achieved / 1e12, "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp64"], "traffic": traffic, "traffic_unit": "bytes per launch",
                     "avg_launch_ms": kernel_ms, "launches_timed": prof["launches"],
                     "timing": "the last step's stage contraction, launches back to back between HIP events",
                     "in_graph_event_bracket_ms": gprof["avg_ms"], "event_pair_latency_ms": gprof["event_latency_ms"],
                     "flops_per_launch": prof["flops"],
                     "algorithmic_bytes_per_launch": prof["bytes"]},
    }
    if not a.no_mixed:
        # mixed forms: FP32 or split-BF16 contractions, FP64 state and stage arithmetic
        forms = {}
        for prec, desc in (("fp32", "FP32 contractions on MFMA (FP32 accumulate), FP64 state"),
                           ("bf16x3", "split-BF16 x3 contractions (FP32 accumulate, FP64 recombination), FP64 state")):
            Sm, _ = make_solver(F, W, torch, weights, prec, stream)
            elm = timed_run(Sm, torch, stream, a.steps, a.warmup)
            pm, _ = contraction_profile(Sm, torch)
            err_long = field_errors(S, Sm, specs)
            # short horizons: fresh runs from the same state
            errs = {}
            for nst in (1, 10):
                S_ref, _ = make_solver(F, W, torch, weights, "fp64", stream)
                S_mix, _ = make_solver(F, W, torch, weights, prec, stream)
                S_ref.advance(5 * nst, sync=True)
                S_mix.advance(5 * nst, sync=True)
                errs["error_vs_fp64_after_%d_steps" % nst] = field_errors(S_ref, S_mix, specs)
                del S_ref, S_mix
            forms[prec] = {"precision": desc, "batched": "hipGraph of whole steps, one contraction launch per stage",
                           "value": npts * 5 * a.steps / elm, "ms_per_step": elm / a.steps * 1e3,
                           "speedup_vs_fp64": el / elm, **errs,
                           "error_vs_fp64_after_%d_steps" % (a.steps + a.warmup + 20): err_long,
                           "contraction_avg_ms": pm["avg_ms"]}
            del Sm
        best = max(forms, key=lambda k: forms[k]["value"])
        out["mixed"] = {"best": best, **forms}
    if not a.no_extras:
        out["derivative_sweep"] = sweep_bench(F, W, torch)
        out["classifier"] = classifier_bench(F, W, torch, weights)
    if not a.no_tiled:
        del S
        out["tiled_channel"] = tiled_channel_run(F, W, torch, weights, a.tiled_steps)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, a.cpu_steps)
    if a.calibration_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
