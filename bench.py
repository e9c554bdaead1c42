"""Benchmark of the FC-SDNN per-stage hot path on one MI355X.

Workload (the large single-GPU configuration): Mach-10 flow past a wedge with
a blunt rear face in the tunnel [0, 1] x [0, 0.5] (15-degree faces, tip at
(0.2, 0.25), rear face at x = 0.4): 244 overlapping subpatches of uneven
sizes (C1 corner subpatches at the tip and the rear corners, skewed-affine
subpatches on the faces, seeded lattice subpatches), 1.15e7 points at
h = 1/4400; SDNN artificial viscosity with a classifier trained on the GPU by
the library's own kernels at set-up; localized smearing of the initial data
in the first step; spectral filter; adaptive step at CFL 0.5.  One benchmark step is one solver time step: viscosity
(classification, smoothing, blend), filter, step size and the five SSPRK
stages (fluxes, grouped FC derivative contractions, viscous terms, update,
boundary conditions, fringe interpolation), replayed as one captured
hipGraph.

Prints one JSON line.  ``value``: point-stage updates/s of the mixed-precision
batched form (split-BF16 contractions with FP32 accumulation and FP64
recombination, FP64 state); ``fp64``: the plain FP64 form on the same
workload and steps; ``fp32``: FP32 contractions.  Per-field max / RMS
differences from the FP64 run after the timed steps, and with the
smoothness classes frozen to the FP64 run's (the precision alone).  The
roofline of the dominant kernel (the grouped stage contraction, timed with
HIP events on the solver stream); the CPU oracle on a bounded sample of the
same workload.
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

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15}
HBM_PEAK = 8.0e12


def log(msg):
    """One progress line on stderr per finished phase of the bench."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the step channel, derivative-sweep and classifier measurements")
    ap.add_argument("--forms", default="bf16x3,fp64,fp32,bf16x6",
                    help="contraction precisions to run on the wedge (the first is the headline value)")
    ap.add_argument("--eager", action="store_true", help="launch kernels one by one instead of replaying step graphs "
                                                           "(for per-dispatch counter runs)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="finish with three plain 256 MiB device copies (byte-counter calibration)")
    ap.add_argument("--stage-variant", default=None,
                    help="pin the stage-contraction tile shape (a kernel name as reported in roofline.kernel) "
                         "instead of tuning it (for counter runs, whose dispatch serialization skews the tuner)")
    ap.add_argument("--tiled", action="store_true",
                    help="also run the tiled step channel at 1.17e7 points (FP64 and split-BF16)")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--classifier-lines", type=int, default=1_000_000,
                    help="synthetic lines for training the classifier (10 %% held out)")
    ap.add_argument("--classifier-epochs", type=int, default=3,
                    help="passes over the training windows (each in a fresh seeded order)")
    return ap.parse_args()


def train_classifier(F, W, torch, nlines=1_000_000, epochs=3, batch=8192, lr=1e-3):
    """Seeded training of the smoothness classifier on the GPU: synthetic
    lines through the solver's FC filter (d = 2, C = 27), 16-point windows,
    class-weighted Adam with the library's training kernels; 10 % of the
    lines held out.  Returns the weights and, on the held-out windows, the
    accuracy and confusion matrix (rows: true class) of the trained network
    and of the modal-decay fallback."""
    t0 = time.perf_counter()
    lines, pos, amp = W.classifier_lines(nlines, seed_salt=51)
    lab = W.window_labels(pos, amp, lines)
    filt = F.lines_apply(torch.tensor(lines, device="cuda"), "filter", 2, 27)
    n = lines.shape[1]
    start = np.clip(np.arange(n) - 8, 0, n - 16)
    idx = torch.tensor(start[:, None] + np.arange(16)[None, :], device="cuda")
    ntrain = nlines - nlines // 10
    wins = filt[:, idx]  # (lines, n, 16)
    labt = torch.tensor(lab, device="cuda")

    def prep(w, y):
        w = w.reshape(-1, 16)
        y = y.reshape(-1)
        lo = w.min(dim=1, keepdim=True).values
        hi = w.max(dim=1, keepdim=True).values
        am = w.abs().max(dim=1, keepdim=True).values
        rng_ = hi - lo
        keep = (rng_ >= 1e-3 * torch.clamp(am, min=1.0)).squeeze(1)
        x = ((w - lo) / torch.where(rng_ > 0, rng_, torch.ones_like(rng_)))[keep].float().contiguous()
        return x, y[keep].int().contiguous(), w, y

    log("classifier data: %d lines, labels and filter done" % nlines)
    x, y, _, _ = prep(wins[:ntrain], labt[:ntrain])
    counts = torch.bincount(y, minlength=3).double()
    cw = (counts.sum() / (3.0 * torch.clamp(counts, min=1.0))).float()
    g = W.rng(4, 52)
    params = torch.tensor(W.sdnn_blob(W.sdnn_init(g)), device="cuda")
    tr = F.SdnnTrainer(params, batch=batch, lr=lr)
    # each epoch reorders the windows once (seeded) and steps through
    # contiguous batches of the reordered copy
    torch.cuda.synchronize()
    t_loop = time.perf_counter()
    gen = torch.Generator().manual_seed(52)
    per_epoch = max(1, y.numel() // batch)
    nsteps = epochs * per_epoch
    for _ in range(epochs):
        perm = torch.randperm(y.numel(), generator=gen).to("cuda")
        xs, ys = x[perm], y[perm]
        for s_ in range(per_epoch):
            tr.step(xs[s_ * batch:(s_ + 1) * batch], ys[s_ * batch:(s_ + 1) * batch], cw)
        del xs, ys, perm
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    loop_s = time.perf_counter() - t_loop
    # held-out lines: raw windows through both classifiers (flat windows are
    # smooth by the classifiers' own rule)
    hw = wins[ntrain:].reshape(-1, 16).contiguous()
    hy = labt[ntrain:].reshape(-1).cpu().numpy()
    ev = {}
    for name, tau in (("sdnn", F.sdnn_infer(params, hw)), ("modal", F.modal_infer(hw))):
        t = tau.cpu().numpy().astype(np.int64)
        conf = np.zeros((3, 3), dtype=np.int64)
        np.add.at(conf, (hy, t), 1)
        ev[name] = {"accuracy": float((t == hy).mean()),
                    "recall_per_class": [float(conf[c, c] / max(conf[c].sum(), 1)) for c in range(3)],
                    "confusion_true_by_predicted": conf.tolist()}
    info = {"lines": nlines, "train_lines": ntrain, "train_windows": int(y.numel()), "batch": batch,
            "steps": nsteps, "epochs": epochs, "train_s": train_s, "train_loop_s": loop_s, "heldout_windows": int(hy.size), **ev}
    return params.cpu().numpy(), info


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
    for prec in ("fp64", "fp32", "bf16x3", "bf16x6"):
        sw = F.DerivSweep(sizes, 4, prec, d=5, C=27)
        sw.autotune(x, d1, d2)
        sw.profile(1)
        for _ in range(10):
            sw.run(x, d1, d2)
        r = sw.profile(-1)
        rate = r["flops"] / (r["avg_ms"] * 1e-3)
        split = prec.startswith("bf16")
        own = PEAK["fp32"] if split else PEAK[prec]
        out[prec] = {"ms": r["avg_ms"], "tflops": rate / 1e12, "frac_of_fp32_peak": rate / PEAK["fp32"],
                     "frac_of_own_peak": rate / own if not split else None,
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


def make_solver(F, W, torch, weights, precision, stream, use_graph=True, specs=None, state=None, av="sdnn",
                smear=False):
    specs = W.step_channel() if specs is None else specs
    prm = F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av=av, filter=True, use_graph=use_graph,
                         precision=precision, sdnn_weights=weights, autotune=True, smear=smear)
    with torch.cuda.stream(stream):
        S = F.Solver(specs, prm, stream=stream)
        w = W.uniform_state(specs, W.STEP_INFLOW) if state is None else state
        for p in range(len(specs)):
            S.set_state(p, w[p])
    return S, specs


def timed_run(S, torch, stream, steps, warmup, retune=True):
    # The first advance tunes the contraction tile on the initial state, where
    # few viscous lines are active; the last warm-up step tunes it again on
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


def _active(specs, p):
    return specs[p].mask if specs[p].mask is not None else np.ones(specs[p].shape, bool)


def field_errors(ref_solver, solver, specs):
    """Per-field max and RMS difference over all active points, relative to
    the field's largest magnitude in the reference run."""
    errs = {}
    for name in ("rho", "mx", "my", "E"):
        ref = np.concatenate([ref_solver.field(p, name)[_active(specs, p)] for p in range(len(specs))])
        got = np.concatenate([solver.field(p, name)[_active(specs, p)] for p in range(len(specs))])
        d = got - ref
        scale = max(np.abs(ref).max(), 1e-300)
        errs[name] = {"max_rel": float(np.abs(d).max() / scale), "rms_rel": float(np.sqrt((d * d).mean()) / scale)}
    return errs


def class_flips(a, b, specs):
    """Points whose smoothness class (either direction) differs between two
    runs' last steps."""
    n = 0
    for p in range(len(specs)):
        m = _active(specs, p)
        for d in ("tau0", "tau1"):
            n += int((a.field(p, d)[m] != b.field(p, d)[m]).sum())
    return n


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


def measured_traffic(kernel, points):
    """HBM bytes of one stage-contraction launch from the counter summary in
    profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's reading),
    if it was taken on this kernel, this workload and the current kernel
    source; None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "wedge_stage_contraction_traffic.json")
    try:
        with open(path) as f:
            m = json.load(f)
        with open(os.path.join(ROOT, m["source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if m.get("kernel") != kernel or m.get("points") != points or m.get("source_sha256") != sha:
        return None
    return {"bytes_per_launch": m["hbm_bytes_per_launch"], "read_bytes": m["hbm_read_bytes_per_launch"],
            "write_bytes": m["hbm_write_bytes_per_launch"],
            "algorithmic_bytes_counted": m["algorithmic_bytes_per_launch"],
            "counted_launches": m.get("counted_state"),
            "vs_algorithmic": m["hbm_bytes_per_launch"] / m["algorithmic_bytes_per_launch"],
            "from": "profiles/wedge_stage_contraction_traffic.md (rocprofv3 FETCH_SIZE x %.3f, WRITE_SIZE x %.3f)"
                    % (m["calibration"]["fetch_factor"], m["calibration"]["write_factor"])}


def roofline_of(prof, precision, kernel):
    """Roofline entries of a stage contraction timed alone: achieved
    algorithmic HBM bytes per second against HBM, and dense MFMA flops
    (2n per point per line operation) against the precision's MFMA peak
    (split BF16: the BF16 peak, three or six products per product)."""
    sec = prof["avg_ms"] * 1e-3
    gbps = prof["bytes"] / sec
    flops = prof["flops"] / sec
    mfma_peak = {"fp64": PEAK["fp64"], "fp32": PEAK["fp32"], "bf16x3": PEAK["bf16"], "bf16x6": PEAK["bf16"]}[precision]
    mfma_rate = flops * {"bf16x3": 3.0, "bf16x6": 6.0}.get(precision, 1.0)
    return {"kernel": kernel, "avg_launch_ms": prof["avg_ms"], "launches_timed": prof["launches"],
            "algorithmic_bytes_per_launch": prof["bytes"], "dense_flops_per_launch": prof["flops"],
            "hbm": {"achieved_GBps": gbps / 1e9, "peak_GBps": HBM_PEAK / 1e9, "frac": gbps / HBM_PEAK},
            "mfma": {"achieved_TFLOPs": mfma_rate / 1e12, "peak_TFLOPs": mfma_peak / 1e12,
                     "frac": mfma_rate / mfma_peak,
                     "fp32_equivalent_frac": flops / PEAK["fp32"]}}


def wedge_run(F, W, torch, weights, forms, steps, warmup, eager=False, stage_variant=None):
    """The wedge tunnel in each contraction precision, from the same initial
    state and for the same steps; the per-field differences from the FP64
    run (after the timed steps, and over 10 steps with the classes frozen to
    the FP64 run's), and each form's stage contraction timed alone."""
    from paper_2506_19370_amd import _lib as L
    specs = W.wedge_tunnel()
    w0 = W.wedge_state(specs)
    npts = int(sum(s.npoints() for s in specs))
    out = {"workload": "Mach-%g wedge tunnel [0,1]x[0,0.5], 15-degree faces, blunt rear face: %d subpatches "
                       "(3 C1 corner, skewed-affine face, rear-face and seeded lattice subpatches, sides 150-300), "
                       "%d points (h = 1/4400), SDNN viscosity (GPU-trained), initial-data smearing, filter, CFL 0.5, "
                       "FC-Gram d=2 C=27"
                       % (W.WEDGE_MACH, len(specs), npts),
           "points": npts, "subpatches": len(specs), "stages_per_step": 5}
    solvers = {}
    for prec in forms:
        stream = torch.cuda.Stream()
        t0 = time.perf_counter()
        S, _ = make_solver(F, W, torch, weights, prec, stream, use_graph=not eager, specs=specs, state=w0, smear=True)
        setup = time.perf_counter() - t0
        if stage_variant:
            S.set_stage_variant(stage_variant)
        el = timed_run(S, torch, stream, steps, warmup, retune=not stage_variant)
        kernel = L.gemm_variant_name(prec, S.stats()["stage_variant"])
        prof, gprof = contraction_profile(S, torch, nsteps=min(20, max(steps, 1)))
        out[prec] = {"value": npts * 5 * steps / el, "ms_per_step": el / steps * 1e3, "host_setup_s": setup,
                     "stage_contraction": roofline_of(prof, prec, kernel),
                     "in_graph_event_bracket_ms": gprof["avg_ms"], "event_pair_latency_ms": gprof["event_latency_ms"]}
        solvers[prec] = (S, stream)
        log("wedge %s: %.3f ms per step, set-up %.1f s" % (prec, out[prec]["ms_per_step"], setup))
    if "fp64" in solvers:
        ref = solvers["fp64"][0]
        nst = steps + warmup + min(20, max(steps, 1))
        for prec in forms:
            if prec == "fp64":
                continue
            out[prec]["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out[prec]["ms_per_step"]
            out[prec]["error_vs_fp64_after_%d_steps" % nst] = field_errors(ref, solvers[prec][0], specs)
            out[prec]["class_flips_vs_fp64_last_step"] = class_flips(ref, solvers[prec][0], specs)
        # the precision alone: both forms from the FP64 run's state, 10 steps
        # with the classes of that state's last step frozen
        state = [ref.cons(p) for p in range(len(specs))]
        tau = [np.stack([ref.field(p, "tau0"), ref.field(p, "tau1")]).astype(np.uint8) for p in range(len(specs))]
        t_now = ref.stats()["t"]
        frozen = {}
        for prec in forms:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                Sf = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="frozen", filter=True,
                                                    precision=prec), stream=stream)
                for p in range(len(specs)):
                    Sf.set_state(p, state[p], prim=False)
                    Sf.set_tau(p, tau[p])
                Sf.set_time(t_now)
                Sf.advance(5 * 10, sync=True)
            frozen[prec] = Sf
        log("wedge frozen-class runs done")
        for prec in forms:
            if prec != "fp64":
                out[prec]["error_vs_fp64_frozen_classes_10_steps"] = field_errors(frozen["fp64"], frozen[prec], specs)
        del frozen
    del solvers
    torch.cuda.synchronize()
    return out


def channel_run(F, W, torch, weights, steps, warmup):
    """The Mach-3 step channel (22 subpatches, 208586 points): FP64 and the
    mixed forms, throughput and speed-up."""
    out = {"workload": "Mach-3 step channel [0,3]x[0,1], step [0.6,3]x[0,0.2], 22 subpatches (C1 L-shaped + C2 "
                       "corner patches), 208586 points, SDNN viscosity, filter, CFL 0.5, FC-Gram d=2 C=27"}
    stream = torch.cuda.Stream()
    for prec in ("fp64", "fp32", "bf16x3"):
        S, specs = make_solver(F, W, torch, weights, prec, stream)
        npts = int(sum(s.npoints() for s in specs))
        el = timed_run(S, torch, stream, steps, warmup)
        out[prec] = {"value": npts * 5 * steps / el, "ms_per_step": el / steps * 1e3}
        del S
    for prec in ("fp32", "bf16x3"):
        out[prec]["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out[prec]["ms_per_step"]
    return out


def tiled_channel_run(F, W, torch, weights, steps, warmup=5):
    """The step channel tiled by 235 subpatches of uneven sizes (1.17e7
    points): FP64 and split-BF16 throughput."""
    specs = W.step_channel_tiled()
    npts = int(sum(s.npoints() for s in specs))
    out = {"workload": "Mach-3 step channel tiled by %d subpatches of sides 150-300, %d points" % (len(specs), npts)}
    for prec in ("fp64", "bf16x3"):
        stream = torch.cuda.Stream()
        S, _ = make_solver(F, W, torch, weights, prec, stream, specs=specs)
        el = timed_run(S, torch, stream, steps, warmup)
        out[prec] = {"value": npts * 5 * steps / el, "ms_per_step": el / steps * 1e3}
        del S
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, weights, steps):
    """The oracle on a bounded sample of the headline workload: the same
    wedge tunnel, Mach number, initial data, SDNN weights, filter and CFL on
    the small decomposition (h = 1/600, 72 subpatches), its first steps
    (set-up not timed), with NumPy/SciPy on the host's cores."""
    from threadpoolctl import threadpool_limits
    from oracle import solver as osolver
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        ncpu = os.cpu_count() or 1
    threads = max(1, min(16, ncpu))
    specs = W.wedge_tunnel(600, 48, 96)
    with threadpool_limits(limits=threads):
        O = osolver.Solver(osolver.patches_from_specs(specs),
                           osolver.Params(fc_d=2, fc_C=27, cfl=0.5, av="sdnn", filter=True, smear=True),
                           sdnn_params=W.sdnn_unblob(weights))
        O.set_prim(W.wedge_state(specs))
        log("oracle set up (%d subpatches)" % len(specs))
        t0 = time.perf_counter()
        for k in range(steps):
            O.step()
            log("oracle step %d" % (k + 1))
        el = time.perf_counter() - t0
    npts = int(sum(s.npoints() for s in specs))
    return {"value": npts * 5 * steps / el, "unit": "point-stage updates/s", "cores": threads, "kind": "oracle",
            "sample": f"wedge tunnel at h = 1/600 ({len(specs)} subpatches, {npts} points; same Mach number, "
                      f"initial data, SDNN weights, filter and CFL as the GPU run), first {steps} steps, "
                      f"FP64 NumPy/SciPy, {el:.1f} s",
            "host": {"nproc": os.cpu_count(), "affinity_cpus": ncpu, "threads_used": threads, "cpu_model": _cpu_model()}}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 (multi-GPU sharding is a design "
                                   "note, not an implemented path)"}))
        sys.exit(2)
    import torch
    import paper_2506_19370_amd as F
    import workloads as W

    forms = [f for f in a.forms.split(",") if f]
    weights, train_info = train_classifier(F, W, torch, nlines=a.classifier_lines, epochs=a.classifier_epochs)
    log("classifier trained on %d lines" % a.classifier_lines)
    wedge = wedge_run(F, W, torch, weights, forms, a.steps, a.warmup, eager=a.eager, stage_variant=a.stage_variant)
    head = forms[0]
    rf = wedge[head]["stage_contraction"]
    dtype = {"bf16x3": "bf16x3+f64", "bf16x6": "bf16x6+f64", "fp32": "f32+f64", "fp64": "f64"}[head]
    out = {
        "metric": "point-stage updates/s, plain FP64 vs mixed-precision batched form at stated error",
        "value": wedge[head]["value"], "unit": "point-stage updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": wedge[head]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": wedge["workload"], "form": head, "points": wedge["points"],
                   "subpatches": wedge["subpatches"], "stages_per_step": 5},
        "roofline": {"bound": "hbm", "kernel": rf["kernel"] + " (grouped FC stage contraction, autotuned tile)",
                     "achieved": rf["hbm"]["achieved_GBps"], "peak": rf["hbm"]["peak_GBps"], "unit": "GB/s",
                     "frac": rf["hbm"]["frac"], "traffic": None,
                     "traffic_detail": None,
                     "achieved_from": "algorithmic bytes of one launch (each operand line the step needs read once "
                                      "in FP64, each derivative written once in the precision of its array) / "
                                      "average launch time",
                     "avg_launch_ms": rf["avg_launch_ms"], "mfma": rf["mfma"],
                     "timing": "the last step's stage contraction, launches back to back between HIP events"},
        "wedge": wedge,
        "classifier_training": train_info,
    }
    tr = measured_traffic(rf["kernel"], wedge["points"])
    if tr is not None:
        out["roofline"]["traffic"] = tr["bytes_per_launch"]
        out["roofline"]["traffic_detail"] = tr
    if not a.no_extras:
        out["step_channel"] = channel_run(F, W, torch, weights, min(a.steps, 2000), a.warmup)
        log("step channel done")
        out["derivative_sweep"] = sweep_bench(F, W, torch)
        log("derivative sweep done")
        out["classifier"] = classifier_bench(F, W, torch, weights)
        log("classifier throughput done")
    if a.tiled:
        out["tiled_channel"] = tiled_channel_run(F, W, torch, weights, a.steps)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, weights, a.cpu_steps)
        log("cpu baseline done")
    if a.calibration_copy:
        # a 256 MiB source written first, then 512 MiB of other writes (so
        # that the source is read from HBM, not from the caches), then three
        # plain copies
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        other = torch.zeros(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        del other
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
