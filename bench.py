"""Benchmark of the STARRED loss+gradient hot path on one MI355X.

One step = one optimiser step of the joint multi-epoch deconvolution: scene
rendering, the fused S_i/D convolution with chi-square, the adjoint and
parameter gradients, the starlet L1 prior and its adjoint, and the Adam update,
on the lensed-quasar workload (100 epochs of 64x64 data, subsampling 2,
128x128 narrow-PSF kernels, 4 point sources, 6 starlet scales). Inputs are
synthetic, seeded, and resident in device memory before the timed region.

Prints one JSON line.
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

PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3


def _make_inputs(prob, plan, torch, seed=0):
    """Noisy synthetic data: the truth rendered and convolved by the device path,
    plus Gaussian background and Poisson noise."""
    from paper_2402_08725_amd import synth
    pt = prob.params_true
    scene = plan.render_scene(pt)
    plan.set_frames(np.zeros(prob.data_size), np.ones(prob.data_size), prob.kernels, prob.W)
    model = plan.convolve_subsample(scene).cpu().numpy().astype(np.float64)
    d, w = synth.add_noise(model, np.random.default_rng(seed))
    plan.set_frames(d, w, prob.kernels, prob.W)
    return d, w


def conv_flops(prob):
    """Algorithmic FP32 flops of one forward launch of the fused S_i + D kernel:
    2 * n_i^2 * (K_i + s - 1)^2 per frame (a multiply and an add per tap)."""
    n = prob.n.astype(np.int64)
    Kp = prob.K.astype(np.int64) + prob.s - 1
    return float(np.sum(2 * n * n * Kp * Kp))


def cpu_baseline(prob_name, budget_s=12.0):
    """The FP64 oracle on a bounded sample of the same workload: the first 8
    epochs of the benchmark problem, repeated until ~budget_s of CPU time."""
    from oracle import oracle as ora
    from paper_2402_08725_amd import synth
    cfg = int(prob_name[-1])
    sample_E = 8
    prob = synth.make_deconv(cfg, E=sample_E)
    rng = np.random.default_rng(0)
    d, w = synth.add_noise(ora.forward_model(prob, prob.params_true), rng)
    p = synth.eval_point(prob, "near", rng)
    t0 = time.perf_counter()
    evals = 0
    while True:
        ora.loss_grad(prob, d, w, p)
        evals += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    eps = evals / el
    return {"value": eps * prob.data_size, "unit": "epoch-px/s", "cores": ora.num_threads(),
            "kind": "oracle",
            "sample": f"{sample_E} of the {prob_name} epochs ({prob.data_size} data px), "
                      f"{evals} FP64 loss+grad evaluations in {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--algo", default="auto", choices=["auto", "direct", "fft"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-baseline comparison")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="also run one plain 256 MiB device copy (memory-counter calibration)")
    args = ap.parse_args()
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
    # the whole run on the plan's stream: no cross-stream ordering per call
    with torch.cuda.stream(plan.stream):
        _run(args, prob, plan, torch, st, synth)


def _run(args, prob, plan, torch, st, synth):
    _make_inputs(prob, plan, torch)
    rng = np.random.default_rng(1)
    p0 = synth.eval_point(prob, "init", rng)
    x = torch.tensor(p0, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(x)
    v = torch.zeros_like(x)
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(x)
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]

    # ---- timed region: optimiser steps (captured graphs of several steps each) ----
    plan.set_graph_mode(not args.no_graph)
    t = 0
    if args.warmup:
        plan.steps(x, m, v, t + 1, lr4, args.warmup, loss_out=loss)
        t += args.warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the K timed steps as one fit (starred_steps: several steps per graph launch)
    plan.steps(x, m, v, t + 1, lr4, args.steps, loss_out=loss)
    t += args.steps
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    value = args.steps / el * prob.data_size

    # ---- fused loss+grad alone vs the plain per-epoch baseline ----
    n_fused = max(20, args.steps // 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_fused):
        plan.loss_grad(x, grad_out=grad, loss_out=loss)
    torch.cuda.synchronize()
    fused_eps = n_fused / (time.perf_counter() - t0)
    plan.set_graph_mode(False)
    plain_eps = None
    if not args.no_plain:
        plan.loss_grad_plain(x, grad_out=grad, loss_out=loss)
        torch.cuda.synchronize()
        n_plain = 5
        t0 = time.perf_counter()
        for _ in range(n_plain):
            plan.loss_grad_plain(x, grad_out=grad, loss_out=loss)
        torch.cuda.synchronize()
        plain_eps = n_plain / (time.perf_counter() - t0)
    if args.copy_calibrate:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        plan.copy_probe(src, dst)
        torch.cuda.synchronize()

    # ---- stage timing (eager launches, HIP events on the launching streams) ----
    n_prof = max(10, min(args.steps, 50))
    plan.set_profiling(True)
    for _ in range(n_prof):
        t += 1
        plan.step(x, m, v, t, lr4, loss_out=loss)
    prof = plan.profile_read()
    plan.set_profiling(False)
    stage_ms = {k: v_["ms"] / max(v_["count"], 1) for k, v_ in prof.items() if v_["count"]}

    # ---- device time of each stage's launches alone (back to back, HIP events) ----
    timed = (["fft_fused", "fft_spec", "fft_mcols", "fft_mrows", "fft_rcols", "fft_acols", "fft_fsum", "fft_arows",
              "spectra", "starlet"] if plan.conv_algo == 2 else ["render", "conv_fwd", "conv_adj", "grad_sums",
                                                                "starlet"])
    kernel_ms = {k: plan.time_stage(x, k, reps=50) for k in timed}
    # stages this plan does not launch (e.g. the line passes when every frame takes the
    # one-launch forward) time as empty event pairs: leave them out of both tables
    idle = {k for k, v_ in kernel_ms.items() if v_ < 5e-4}
    kernel_ms = {k: v_ for k, v_ in kernel_ms.items() if k not in idle}
    stage_ms = {k: v_ for k, v_ in stage_ms.items() if k not in idle}
    roof = roofline(prob, plan, kernel_ms)
    out = {
        "metric": "loss+grad evals/s (epoch-pixels/s), fused vs plain, grad rel err <=1e-4",
        "value": value, "unit": "epoch-px/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{prob.name}: {prob.E} epochs of {int(prob.n[0])}x{int(prob.n[0])} "
                               f"data, s={prob.s}, {int(prob.K[0])}x{int(prob.K[0])} kernels, "
                               f"M={prob.M}, J={prob.J}",
                   "epochs": prob.E, "data_px_per_eval": prob.data_size,
                   "conv_algo": {1: "direct", 2: "fft"}.get(plan.conv_algo, "?"),
                   "graph": not args.no_graph},
        "evals_per_s_step": args.steps / el,
        "fused_vs_plain": ({"fused_loss_grad_evals_per_s": fused_eps,
                            "plain_loss_grad_evals_per_s": plain_eps,
                            "fused_epoch_px_per_s": fused_eps * prob.data_size,
                            "plain_epoch_px_per_s": plain_eps * prob.data_size,
                            "speedup": fused_eps / plain_eps} if plain_eps else None),
        "stage_ms_per_step": {k: round(v_, 4) for k, v_ in stage_ms.items()},
        "stage_device_ms": {k: round(v_, 4) for k, v_ in kernel_ms.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob.name)
    print(json.dumps(out), flush=True)


def roofline(prob, plan, stage_ms):
    """Roofline of the dominant kernel, from its average device duration (its
    launches timed back to back with HIP events on the plan's stream)."""
    if plan.conv_algo == 1:
        fwd_ms = stage_ms["conv_fwd"]
        flops = conv_flops(prob)
        achieved = flops / (fwd_ms * 1e-3) / 1e12
        return {"bound": "alu", "kernel": "k_fwd_direct (fused S_i + D + residual + chi2)",
                "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": None,
                "avg_launch_ms": round(fwd_ms, 4), "algorithmic_flops": flops}
    # FFT path: the slowest pass, against the HBM peak with its algorithmic bytes (at
    # these sizes the passes are VALU- and latency-bound, so the fraction stays low)
    alg = fft_kernel_bytes(prob)
    name = max((k for k in alg if k in stage_ms), key=lambda k: stage_ms[k])
    ms = stage_ms[name]
    by = alg[name]
    achieved = by / (ms * 1e-3) / 1e9
    traffic = committed_traffic(FFT_KERNEL_NAMES[name])
    return {"bound": "hbm", "kernel": FFT_KERNEL_NAMES[name], "stage": name,
            "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "avg_launch_ms": round(ms, 4), "algorithmic_bytes": by}


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
}


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed memory-counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "fft_pass_traffic_cfg2.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != _sources_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(kernel.split(" ")[0])


def _sources_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("starred_fft.hip", "starred_fft.h"):
        with open(os.path.join(ROOT, "paper_2402_08725_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def fft_kernel_bytes(prob):
    """Algorithmic bytes of each FFT-path launch for the whole batch: what each
    pass must read and write once (complex64 spectra, FP32 images)."""
    tot = {k: 0 for k in FFT_KERNEL_NAMES}
    fused_classes = set()
    for n, K in zip(prob.n, prob.K):
        n = int(n)
        F = prob.s * n
        P = _good(F + int(K) // 2, prob.s)
        Q = P // prob.s
        HP, HQ = P // 2 + 1, Q // 2 + 1
        s2 = prob.s * prob.s
        tot["fft_acols"] += 8 * (P * HP + Q * HQ)      # kernel spectrum and rho_hat read once
        if _fused(Q, n, P, prob.M):
            # kernel spectrum, data and weights in, rho_hat out; the class's h spectrum once
            tot["fft_fused"] += 8 * P * HP + 8 * n * n + 8 * Q * HQ
            if (n, int(K)) not in fused_classes:
                fused_classes.add((n, int(K)))
                tot["fft_fused"] += 8 * P * HP
            continue
        tot["fft_spec"] += 8 * (s2 * Q * HQ + Q * HQ)
        tot["fft_mcols"] += 8 * (Q * HQ + n * HQ)
        tot["fft_mrows"] += 8 * (2 * n * HQ) + 8 * n * n
        tot["fft_rcols"] += 8 * (n * HQ + Q * HQ)
    Q3 = 1 + 3 * prob.M
    npb = {int(P_): nrr for _, P_, _, nrr in _classes(prob)}
    for n, K in zip(prob.n, prob.K):
        P = _good(prob.s * int(n) + int(K) // 2, prob.s)
        tot["fft_fsum"] += 8 * (npb[P] * Q3 + Q3)       # block dot-product partials in, frame sums out
    for F_, P_, nch, _ in _classes(prob):
        HP_ = P_ // 2 + 1
        # the class's summed adjoint spectrum leaves once (the frame-chunk partial
        # spectra and their re-read are the implementation's, not the algorithm's)
        tot["fft_acols"] += 8 * P_ * HP_
        tot["fft_arows"] += 8 * (P_ * HP_ + 2 * F_ * HP_) + 4 * F_ * F_
    return {k: float(v) for k, v in tot.items()}


def _fused(Q, n, P, M):
    """Whether frames of this shape take the one-launch forward: its two LDS planes of
    max(Q/2+1, n) lines of Q+1 complex values, the Q twiddles and the (1+4M) P table
    values fit in 150 KiB."""
    return (2 * max(Q // 2 + 1, n) * (Q + 1) + Q + (1 + 4 * M) * P) * 8 <= 150 * 1024


ADJ_FRAMES = 2  # frames per work group of the frequency-domain adjoint (kAdjFrames)


def _classes(prob):
    """(F, P, frame chunks, row ranges) of each shape class, as the plan groups them
    for the frequency-domain adjoint (chunks of ADJ_FRAMES frames, about 512 work groups)."""
    out = {}
    for n, K in zip(prob.n, prob.K):
        key = (int(n), int(K))
        out[key] = out.get(key, 0) + 1
    nchunks = sum((ncf + ADJ_FRAMES - 1) // ADJ_FRAMES for ncf in out.values())
    res = []
    for (n, K), ncf in out.items():
        F = prob.s * n
        P = _good(F + K // 2, prob.s)
        HP = P // 2 + 1
        CX = 64 if HP <= 64 else (128 if HP <= 128 else 256)
        RG = 256 // CX
        want = max(1, (512 + nchunks - 1) // nchunks)
        arr = (P + want - 1) // want
        arr = min(64, max(4 * RG, ((arr + RG - 1) // RG) * RG))
        res.append((F, P, (ncf + ADJ_FRAMES - 1) // ADJ_FRAMES, (P + arr - 1) // arr))
    return res


def _good(need, s):
    P = need
    while True:
        if P % (2 * s) == 0:
            r = P
            for f in (2, 3, 5):
                while r % f == 0:
                    r //= f
            if r == 1:
                return P
        P += 1


if __name__ == "__main__":
    main()
