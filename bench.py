"""Benchmark of the STARRED loss+gradient hot path on one MI355X.

One step = one optimiser step of the joint multi-epoch deconvolution: scene
rendering, the fused S_i/D convolution with chi-square, the adjoint and
parameter gradients, the starlet L1 prior and its adjoint, and the Adam update.
The default workload is the supernova time series: 1000 epochs with ragged
stamp sides drawn from {32, 48, 64, 96, 128}, subsampling 2, a 256x256 host
grid, kernels of side min(2n, 128), one transient point source and 6 starlet
scales whose weights come from Monte Carlo noise propagation (Sec. 2.3).
Inputs are synthetic, seeded, and resident in device memory before the timed
region.

Timing: W untimed warm-up steps, then every captured graph the timed call uses
is built (capture steps, reported), then exactly K steps are timed between two
device synchronisations (`value`, `ms_per_step`). A longer series of graph
launches, each between two HIP events on the plan's stream, gives the median
and p10/p90 per step, and the loss+gradient evaluation alone (fused) against
the plain per-epoch kernels.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3
STEPS_PER_GRAPH = 8  # optimiser steps per graph launch of starred_steps
METRIC = "loss+grad evals/s (epoch-pixels/s), fused vs plain, grad rel err <=1e-4"


def _pct(xs):
    a = np.asarray(xs, dtype=np.float64)
    return {"median": float(np.median(a)), "p10": float(np.percentile(a, 10)),
            "p90": float(np.percentile(a, 90)), "n": int(a.size)}


def _make_inputs(prob, plan, seed=0):
    """Noisy synthetic data: the truth rendered and convolved by the device path,
    plus Gaussian background and Poisson noise; W by Monte Carlo noise propagation
    through frame 0 (64 realizations, per scale, coarse plane not penalised)."""
    from paper_2402_08725_amd import synth
    pt = prob.params_true
    scene = plan.render_scene(pt)
    plan.set_frames(np.zeros(prob.data_size), np.ones(prob.data_size), prob.kernels, prob.W)
    model = plan.convolve_subsample(scene).cpu().numpy().astype(np.float64)
    d, w = synth.add_noise(model, np.random.default_rng(seed))
    plan.set_frames(d, w, prob.kernels, prob.W)
    n0 = int(prob.n[0])
    W = plan.noise_weights(1.0 / w[:n0 * n0], 64, seed=1000 + seed, per_pixel=False, frame=0)
    W = W.cpu().numpy().astype(np.float64)
    W[-1] = 0.0
    W = synth.f32(W)
    t0 = time.perf_counter()
    plan.set_frames(d, w, prob.kernels, W)  # with the automatic choice: the autotuner runs here
    tune_s = time.perf_counter() - t0
    return d, w, W, tune_s


# --------------------------------------------------------------------------- #
# Algorithmic bytes (per launch) of each kernel, from per-unit figures         #
# --------------------------------------------------------------------------- #
# Per frame i (data side n, kernel side K), FP32 values read or written once:
#   data d_i and inverse variance w_i: 8 n^2;  kernel s_i: 4 K^2;
#   weighted residual rho_i (produced by the forward, consumed by the adjoint): 4 n^2.
# Per shape class c (fine window side F): its window of h read once (4 F^2), its
# window of dL/dh written once (4 F^2). Passes that only move the transforms'
# intermediate spectra have no algorithmic bytes of their own.

def fft_kernel_bytes(prob, fused_classes, keep=None):
    """Algorithmic bytes per launch of each FFT-path kernel for the whole batch.
    fused_classes: set of (n, K) whose frames take the one-launch forward; keep: mask of
    the frames on the FFT algorithm (all when None)."""
    tot = {k: 0.0 for k in FFT_KERNEL_NAMES}
    classes = set()
    for i, (n, K) in enumerate(zip(prob.n.tolist(), prob.K.tolist())):
        if keep is not None and not keep[i]:
            continue
        classes.add((n, K))
        if (n, K) in fused_classes:
            tot["fft_fused"] += 8 * n * n + 4 * K * K + 4 * n * n
        else:
            tot["fft_spec"] += 4 * K * K
            tot["fft_mrows"] += 8 * n * n + 4 * n * n
        tot["fft_acols"] += 4 * K * K + 4 * n * n
    for n, K in classes:
        F = prob.s * n
        tot["spectra"] += 4 * F * F
        tot["fft_arows"] += 4 * F * F
    return tot


FFT_KERNEL_NAMES = {
    "fft_fused": "k_frame_fwd (one-launch forward per frame: spectral product, inverse 2-D transform, "
                 "residual, chi-square, forward 2-D transform of rho)",
    "fft_spec": "k_spec_fwd (spectral product and alias fold)",
    "fft_mcols": "k_lines<OpMCols> (inverse columns of the model spectra)",
    "fft_mrows": "k_fwd_rows (inverse rows, residual, chi-square, rho row spectra)",
    "fft_rcols": "k_lines<OpRhoCols> (forward columns of rho)",
    "fft_acols": "k_spec_adj (adjoint spectral products summed over frames, Parseval dot products)",
    "fft_arows": "k_lines<OpGCols/OpGRows> (inverse transform of the summed adjoint spectra)",
    "fft_fsum": "k_adj_sums (sum of the frame-chunk spectra; per-frame sums of the block dot products)",
    "spectra": "k_lines<OpHRows/OpHCols> (spectra of the h windows and the source tables)",
}


def direct_flops(prob, sel=None):
    """Algorithmic FP32 flops of one launch of the fused S_i + D kernel (or of its
    adjoint, which applies the same taps): 2 n_i^2 (K_i + s - 1)^2 per frame (a
    multiply and an add per tap), over the frames sel (all when None)."""
    n = prob.n.astype(np.int64)
    Kp = prob.K.astype(np.int64) + prob.s - 1
    f = 2 * n * n * Kp * Kp
    return float(np.sum(f if sel is None else f[sel]))


def roofline(prob, plan, stage_ms, x):
    """Roofline of the dominant kernel of a step (the stage with the longest in-step
    duration: HIP events around each launch on the plan's stream, from the profiled
    steps): its algorithmic bytes (or flops) per launch over its average launch
    duration, timed as 50 launches back to back between two HIP events on the plan's
    stream (what a kernel trace reports per dispatch; the in-step interval also holds
    the event and dispatch gap). Frames of classes on the direct algorithm count for
    the direct kernels, the others for the FFT kernels."""
    cls = plan.classes()
    direct = {(c["n"], c["K"]) for c in cls if c["algo"] == 1}
    fused = {(c["n"], c["K"]) for c in cls if c["algo"] == 2 and c["fused"]}
    cand = [k for k in list(FFT_KERNEL_NAMES) + ["direct_fwd", "direct_adj"] if k in stage_ms]
    name = max(cand, key=lambda k: stage_ms[k])
    in_step_ms = stage_ms[name]
    ms = plan.time_stage(x, name, reps=50)
    if name in ("direct_fwd", "direct_adj"):
        sel = np.array([(n, K) in direct for n, K in zip(prob.n.tolist(), prob.K.tolist())])
        flops = direct_flops(prob, sel)
        achieved = flops / (ms * 1e-3) / 1e12
        kern = ("k_fwd_direct (fused S_i + D + residual + chi2)" if name == "direct_fwd"
                else "k_adj_direct (S_i^T D^T, s^2 phase correlations)")
        return {"bound": "alu", "kernel": kern, "stage": name,
                "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": None,
                "avg_launch_ms": round(ms, 4), "in_step_ms": round(in_step_ms, 4), "algorithmic_flops": flops}
    keep = np.array([(n, K) not in direct for n, K in zip(prob.n.tolist(), prob.K.tolist())])
    alg = fft_kernel_bytes(prob, fused, keep)
    by = alg[name]
    achieved = by / (ms * 1e-3) / 1e9
    traffic = committed_traffic(prob.name, FFT_KERNEL_NAMES[name].split(" ")[0])
    return {"bound": "hbm", "kernel": FFT_KERNEL_NAMES[name], "stage": name,
            "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "traffic_source": ("rocprofv3 FETCH_SIZE/WRITE_SIZE per launch (committed counter summary of "
                               "the same sources)" if traffic else None),
            "avg_launch_ms": round(ms, 4), "in_step_ms": round(in_step_ms, 4), "algorithmic_bytes": by,
            "traffic_frac": round(traffic / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4) if traffic else None}


def committed_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed memory-counter summary of
    this workload, or None when the sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"fft_pass_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != sources_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(kernel)


def write_traffic(workload, fetch_dir, write_dir):
    """Write profiles/fft_pass_traffic_<workload>.json from two rocprofv3 --pmc runs of
    this script with --copy-calibrate (FETCH_SIZE, then WRITE_SIZE; csv output): HBM bytes
    per launch of each kernel's most frequent launch shape, FETCH_SIZE and WRITE_SIZE (KiB)
    scaled by what they read for the 256 MiB copy kernel, stamped with the sources' hash.
    Prints the per-kernel rows."""
    import csv
    import collections
    import statistics

    def load(d, cname):
        by = collections.defaultdict(list)
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != cname:
                    continue
                n = r["Kernel_Name"].replace("void ", "").replace("starred::", "").split("(")[0]
                by[(n, int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        return by
    F, W = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_kib = 256 * 1024
    fc = statistics.median(F[next(k for k in F if k[0] == "k_copy_probe")])
    wc = statistics.median(W[next(k for k in W if k[0] == "k_copy_probe")])
    fs, ws = copy_kib / fc, copy_kib / wc
    best = {}
    for (n, g), v in F.items():
        if n not in best or len(v) > len(F[(n, best[n])]):
            best[n] = g
    per = {}
    print(f"FETCH scale {fs:.4f} (copy {fc:.0f} KiB), WRITE scale {ws:.4f} (copy {wc:.0f} KiB)")
    for n in sorted(best):
        g = best[n]
        f_ = statistics.median(F[(n, g)])
        w_ = statistics.median(W.get((n, g), [float("nan")]))
        b = (f_ * fs + w_ * ws) * 1024
        per[n] = b
        per[n.split("<")[0]] = b
        print(f"| `{n}` | {g} | {len(F[(n, g)])} | {f_:.1f} | {w_:.1f} | {b / 1e6:.3f} |")
    rec = {"workload": workload, "source_sha256": sources_hash(), "fetch_scale": fs, "write_scale": ws,
           "bytes_per_launch": per}
    with open(os.path.join(ROOT, "profiles", f"fft_pass_traffic_{workload}.json"), "w") as f:
        json.dump(rec, f, indent=1)


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2402_08725_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(prob_name, budget_s=12.0):
    """The FP64 oracle on a bounded sample of the same workload: its first 8 epochs
    (all threads, repeated for about budget_s) and its first 2 epochs on one thread."""
    from oracle import oracle as ora
    from paper_2402_08725_amd import synth
    full = synth.make_deconv(int(prob_name[-1]))
    out = {}
    for label, nfr, threads, budget in (("all", 8, 0, budget_s), ("one", 2, 1, 4.0)):
        prob = synth.subset(full, range(nfr))
        rng = np.random.default_rng(0)
        ora.set_num_threads(threads)
        d, w = synth.add_noise(ora.forward_model(prob, prob.params_true), rng)
        p = synth.eval_point(prob, "near", rng)
        t0 = time.perf_counter()
        evals = 0
        while True:
            ora.loss_grad(prob, d, w, p)
            evals += 1
            el = time.perf_counter() - t0
            if el >= budget:
                break
        out[label] = (evals / el * prob.data_size, ora.num_threads(), evals, el, prob)
    ora.set_num_threads(0)
    v, cores, evals, el, prob = out["all"]
    v1, _, evals1, el1, prob1 = out["one"]
    return {"value": v, "unit": "epoch-px/s", "cores": cores, "kind": "oracle",
            "sample": f"epochs 0-7 of {prob_name} (sides {prob.n.tolist()}, {prob.data_size} data px): "
                      f"{evals} FP64 loss+grad evaluations in {el:.1f} s on {cores} threads",
            "one_thread": {"value": v1, "unit": "epoch-px/s",
                           "sample": f"epochs 0-1 (sides {prob1.n.tolist()}, {prob1.data_size} data px): "
                                     f"{evals1} evaluations in {el1:.1f} s"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


# --------------------------------------------------------------------------- #

def _event_series(torch, fn, min_calls, min_s, max_calls=100000):
    """Milliseconds of each fn() call between two HIP events on the current stream
    (the plan's), until at least min_calls calls and min_s seconds."""
    out = []
    t0 = time.perf_counter()
    while len(out) < max_calls:
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
        if len(out) >= min_calls and time.perf_counter() - t0 >= min_s:
            break
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="cfg4")
    ap.add_argument("--algo", default="auto", choices=["auto", "direct", "fft"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-baseline comparison")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--stats-s", type=float, default=1.0, help="least seconds of each event series")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="also run one plain 256 MiB device copy (memory-counter calibration)")
    ap.add_argument("--prior-late", type=int, default=None,
                    help="pin the starlet prior's placement after tuning (set_fft_shapes prior_late)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the committed traffic record of --config from two rocprofv3 --pmc "
                         "runs (FETCH_SIZE, WRITE_SIZE) and exit (no GPU)")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.config, *args.write_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2402_08725_amd import starred as st
    from paper_2402_08725_amd import synth

    cfg = int(args.config[-1])
    prob = synth.make_deconv(cfg)
    algo = {"auto": st.CONV_AUTO, "direct": st.CONV_DIRECT, "fft": st.CONV_FFT}[args.algo]
    plan = st.Plan.for_problem(prob, conv_algo=algo)
    # the whole run on the plan's stream: no cross-stream ordering per call, and
    # torch's events are recorded on the stream the kernels run on
    with torch.cuda.stream(plan.stream):
        out = _run(args, prob, plan, torch, st, synth)
        extra = {} if args.no_extra else _extra_workloads(args, torch, st, synth)
    if extra:
        out["other_workloads"] = extra
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob.name)
    print(json.dumps(out), flush=True)


def _run(args, prob, plan, torch, st, synth):
    _, _, W, tune_s = _make_inputs(prob, plan)
    if args.prior_late is not None:
        # (counter runs: kernels serialised by the profiler can tip the tuner's choice of
        # the prior's placement; pinning it keeps the launches those of the timed runs)
        plan.set_fft_shapes(prior_late=args.prior_late)
    rng = np.random.default_rng(1)
    p0 = synth.eval_point(prob, "init", rng)
    x = torch.tensor(p0, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(x)
    v = torch.zeros_like(x)
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(x)
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    graph = not args.no_graph

    # ---- warm-up, then the graphs the timed call replays (captured before t0) ----
    plan.set_graph_mode(graph)
    t = 0
    if args.warmup:
        plan.steps(x, m, v, t + 1, lr4, args.warmup, loss_out=loss)
        t += args.warmup
    capture = 0
    if graph:
        shapes = set()
        if args.warmup >= STEPS_PER_GRAPH:
            shapes.add(STEPS_PER_GRAPH)
        if args.warmup % STEPS_PER_GRAPH:
            shapes.add(1)
        for need, n in ((args.steps >= STEPS_PER_GRAPH, STEPS_PER_GRAPH), (args.steps % STEPS_PER_GRAPH > 0, 1)):
            if need and n not in shapes:
                plan.steps(x, m, v, t + 1, lr4, n, loss_out=loss)
                t += n
                capture += n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # ---- timed region: exactly K steps as one fit ----
    plan.steps(x, m, v, t + 1, lr4, args.steps, loss_out=loss)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t += args.steps
    ms = el * 1e3 / args.steps
    value = args.steps / el * prob.data_size

    # ---- per-step distribution: graph launches of STEPS_PER_GRAPH steps each ----
    def launch_steps():
        nonlocal t
        plan.steps(x, m, v, t + 1, lr4, STEPS_PER_GRAPH, loss_out=loss)
        t += STEPS_PER_GRAPH
    series = _event_series(torch, launch_steps, max(1, 200 // STEPS_PER_GRAPH), args.stats_s)
    step_stats = _pct([s / STEPS_PER_GRAPH for s in series])

    # ---- fused loss+grad alone vs the plain per-epoch baseline ----
    plan.loss_grad(x, grad_out=grad, loss_out=loss)
    fser = _event_series(torch, lambda: plan.loss_grad(x, grad_out=grad, loss_out=loss), 200, args.stats_s)
    fused = _pct(fser)
    plan.set_graph_mode(False)
    plain = None
    if not args.no_plain:
        plan.loss_grad_plain(x, grad_out=grad, loss_out=loss)
        torch.cuda.synchronize()
        pser = _event_series(torch, lambda: plan.loss_grad_plain(x, grad_out=grad, loss_out=loss), 3, 0.0)
        plain = _pct(pser)
    if args.copy_calibrate:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        plan.copy_probe(src, dst)
        torch.cuda.synchronize()

    # ---- per-kernel device time inside eager steps (HIP events around each launch) ----
    n_prof = 20
    plan.set_profiling(True)
    for _ in range(n_prof):
        t += 1
        plan.step(x, m, v, t, lr4, loss_out=loss)
    prof = plan.profile_read()
    plan.set_profiling(False)
    stage_ms = {k: v_["ms"] / max(v_["count"], 1) for k, v_ in prof.items() if v_["count"]}
    # stages with no work in this plan (their event pairs only time the dispatch gap)
    cls = plan.classes()
    idle = {k for k, v_ in stage_ms.items() if v_ < 5e-4}
    if not any(c["algo"] == 2 and not c["fused"] for c in cls):
        idle |= {"fft_spec", "fft_mcols", "fft_mrows", "fft_rcols"}
    if not any(c["algo"] == 1 for c in cls):
        idle |= {"direct_fwd", "direct_adj", "render", "grad_sums"}
    stage_ms = {k: v_ for k, v_ in stage_ms.items() if k not in idle}
    roof = roofline(prob, plan, stage_ms, x)
    b_alg = step_alg_bytes(prob, W)
    fused_ms = fused["median"]
    out = {
        "metric": METRIC,
        "value": value, "unit": "epoch-px/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload_name(prob),
                   "epochs": prob.E, "data_px_per_eval": prob.data_size, "fine_px_per_eval": prob.fine_size,
                   "conv_algo": {1: "direct", 2: "fft"}.get(plan.conv_algo, "?"),
                   "graph": graph},
        "capture_steps": capture,
        "step_ms": {k: (round(v_, 5) if isinstance(v_, float) else v_) for k, v_ in step_stats.items()},
        "fine_epoch_px_per_s": args.steps / el * prob.fine_size,
        "autotune": autotune_summary(plan, tune_s),
        "fused_vs_plain": {
            "fused_loss_grad_ms": {k: (round(v_, 5) if isinstance(v_, float) else v_) for k, v_ in fused.items()},
            "fused_epoch_px_per_s": prob.data_size / (fused_ms * 1e-3),
            "plain_loss_grad_ms": ({k: (round(v_, 4) if isinstance(v_, float) else v_) for k, v_ in plain.items()}
                                   if plain else None),
            "plain_epoch_px_per_s": (prob.data_size / (plain["median"] * 1e-3)) if plain else None,
            "speedup": (plain["median"] / fused_ms) if plain else None},
        "stage_ms_per_step": {k: round(v_, 4) for k, v_ in stage_ms.items()},
        "roofline": roof,
        "step_literal_hbm": {"algorithmic_bytes": b_alg,
                             "frac": round(b_alg / (step_stats["median"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
    }
    return out


def autotune_summary(plan, tune_s):
    """The autotuner's choices per shape class and the time it took (excluded from the
    timed steps; reported as the counterpart of a compile step)."""
    info = plan.autotune_info()
    names = {0: "direct", 1: "fft-fused", 2: "fft-lines"}
    cls = []
    for c in plan.classes():
        choice = "direct" if c["algo"] == 1 else ("fft-fused" if c["fused"] else "fft-lines")
        cls.append({"n": c["n"], "K": c["K"], "frames": c["n_frames"], "P": c["P"], "choice": choice,
                    "tried_ms": {names[k]: round(v, 4) for k, v in enumerate(c["tune_ms"]) if v >= 0}})
    return {"tune_ms": round(info["wall_ms"], 2), "cached": info["cached"], "set_frames_s": round(tune_s, 3),
            "adj_blocks": info["adj_blocks"], "adj_frames": info["adj_frames"], "line_groups": info["line_groups"],
            "split_forward": info["split_forward"], "prior_late": info["prior_late"], "classes": cls}


def step_alg_bytes(prob, W):
    """Bytes an evaluation must move: d_i, w_i, s_i and the per-frame parameters once,
    h read once, dL/dh written once, W."""
    n = prob.n.astype(np.int64)
    K = prob.K.astype(np.int64)
    NN = prob.N * prob.N
    return float(8 * np.sum(n * n) + 4 * np.sum(K * K) + 4 * 2 * (prob.E + prob.E * prob.M)
                 + 8 * NN + 4 * np.size(W))


def workload_name(prob):
    sides = sorted(set(prob.n.tolist()))
    ks = sorted(set(prob.K.tolist()))
    side = (f"{sides[0]}x{sides[0]}" if len(sides) == 1 else "ragged " + "/".join(map(str, sides)))
    kern = (f"{ks[0]}x{ks[0]}" if len(ks) == 1 else "min(2n,128) " + "/".join(map(str, ks)))
    return (f"{prob.name}: {prob.E} epochs of {side} data, s={prob.s}, {prob.N}x{prob.N} grid, {kern} kernels, "
            f"M={prob.M}, J={prob.J}")


def _extra_workloads(args, torch, st, synth):
    """The other workloads, each a short graph-mode fit: median and p10/p90 per step."""
    res = {}
    for cfg in (5, 2, 1):
        prob = synth.make_deconv(cfg)
        plan = st.Plan.for_problem(prob)
        with torch.cuda.stream(plan.stream):
            _make_inputs(prob, plan)
            x = torch.tensor(synth.eval_point(prob, "init", np.random.default_rng(1)), dtype=torch.float32,
                             device="cuda")
            m = torch.zeros_like(x)
            v = torch.zeros_like(x)
            loss = torch.empty(3, dtype=torch.float64, device="cuda")
            lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
            plan.set_graph_mode(True)
            tt = [0]

            def go():
                plan.steps(x, m, v, tt[0] + 1, lr4, STEPS_PER_GRAPH, loss_out=loss)
                tt[0] += STEPS_PER_GRAPH
            for _ in range(3):
                go()
            ser = _pct([s / STEPS_PER_GRAPH for s in _event_series(torch, go, 25, 0.3)])
        res[prob.name] = {"workload": workload_name(prob), "conv_algo": {1: "direct", 2: "fft"}[plan.conv_algo],
                          "step_ms": {k: (round(v_, 5) if isinstance(v_, float) else v_) for k, v_ in ser.items()},
                          "epoch_px_per_s": prob.data_size / (ser["median"] * 1e-3)}
        plan.close()
    # per-frame shifts and rotations (the lensed-quasar shapes): each frame rendered under
    # its transform and convolved by the faster of the direct kernels and its own
    # spectrum (timed at set_frame_transforms), the transforms' gradient written too
    prob = synth.make_deconv(2)
    plan = st.Plan.for_problem(prob)
    with torch.cuda.stream(plan.stream):
        _make_inputs(prob, plan)
        rng = np.random.default_rng(7)
        xf = np.stack([rng.uniform(-2, 2, prob.E), rng.uniform(-2, 2, prob.E), rng.uniform(-0.02, 0.02, prob.E)], 1)
        xf_d = torch.tensor(xf, dtype=torch.float32, device="cuda")
        gxf = torch.empty_like(xf_d)
        plan.set_frame_transforms(xf_d, grad_out=gxf)
        xalgo, xms = plan.frame_transforms_info()
        x = torch.tensor(synth.eval_point(prob, "init", np.random.default_rng(1)), dtype=torch.float32, device="cuda")
        m = torch.zeros_like(x)
        v = torch.zeros_like(x)
        loss = torch.empty(3, dtype=torch.float64, device="cuda")
        lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
        plan.set_graph_mode(True)
        tt = [0]

        def go_xf():
            plan.steps(x, m, v, tt[0] + 1, lr4, STEPS_PER_GRAPH, loss_out=loss)
            tt[0] += STEPS_PER_GRAPH
        for _ in range(2):
            go_xf()
        ser = _pct([s / STEPS_PER_GRAPH for s in _event_series(torch, go_xf, 10, 0.3)])
    res["cfg2_transforms"] = {"workload": workload_name(prob) + ", per-frame shifts and rotations",
                              "conv_algo": {1: "direct", 2: "fft"}.get(xalgo, "none"),
                              "choice_ms_per_eval": {k: round(v_, 4) for k, v_ in xms.items()},
                              "step_ms": {k: (round(v_, 5) if isinstance(v_, float) else v_) for k, v_ in ser.items()},
                              "epoch_px_per_s": prob.data_size / (ser["median"] * 1e-3)}
    plan.close()
    # PSF mode (star stamps): one step = loss, gradient and update of (eta_M, b, a, c)
    pp = synth.make_psf(3)
    plan = st.Plan.for_psf(pp)
    with torch.cuda.stream(plan.stream):
        from paper_2402_08725_amd import synth as sy
        model = plan.psf_model(pp.params_true).cpu().numpy().astype(np.float64)
        d, w = sy.add_noise(model, np.random.default_rng(3), poisson=False)
        plan.set_frames(d, w, None, pp.W)
        x = torch.tensor(sy.psf_eval_point(pp, "near", np.random.default_rng(4)), dtype=torch.float32,
                         device="cuda")
        m = torch.zeros_like(x)
        v = torch.zeros_like(x)
        loss = torch.empty(3, dtype=torch.float64, device="cuda")
        plan.set_graph_mode(True)
        tt = [0]

        def go():
            plan.steps(x, m, v, tt[0] + 1, [1e-4, 1e-6, 10.0, 0.01], STEPS_PER_GRAPH, loss_out=loss)
            tt[0] += STEPS_PER_GRAPH
        for _ in range(3):
            go()
        ser = _pct([s / STEPS_PER_GRAPH for s in _event_series(torch, go, 25, 0.3)])
    res["cfg3"] = {"workload": f"cfg3 (PSF mode): {pp.S} star stamps of {pp.n}x{pp.n}, s={pp.s}, "
                               f"{pp.N}x{pp.N} PSF grid, J={pp.J}",
                   "step_ms": {k: (round(v_, 5) if isinstance(v_, float) else v_) for k, v_ in ser.items()},
                   "epoch_px_per_s": pp.data_size / (ser["median"] * 1e-3)}
    plan.close()
    return res


if __name__ == "__main__":
    main()
