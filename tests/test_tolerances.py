"""Where a parity bar is wider than the bar on one evaluation, the reason is pinned
here, on the CPU, with the oracle alone.

The 200-step Adam comparison (cfg1 shapes, Adam of Sec. 3's runs) compares the end
of two trajectories, not one evaluation. The l1 term of Eq. 6 has a subgradient
that jumps where a starlet coefficient crosses zero, so a gradient error far below
the one-evaluation bar can move a crossing by a step and send the run on a nearby
but different path. The test perturbs the oracle's own FP64 gradients by relative
errors of 1e-6 (the size of the FP32 path's gradient error) and measures how far
the final loss moves: already above 1e-4, below the 1e-3 bar of the GPU test.
"""
import numpy as np

from oracle import oracle as ora
from paper_2402_08725_amd import synth

PERTURB = 1e-6
ADAM200_LOSS_BAR = 1e-3


def _adam_run(prob, d, w, p0, noise_seed):
    lrv = prob.lr_vector()
    po = p0.copy()
    mo = np.zeros_like(po)
    vo = np.zeros_like(po)
    r = None if noise_seed is None else np.random.default_rng(noise_seed)
    for t in range(1, 201):
        _, go = ora.loss_grad(prob, d, w, po)
        if r is not None:
            go = go * (1.0 + PERTURB * r.standard_normal(go.shape))
        ora.adam_step(po, go, mo, vo, t, lrv)
    lo, _ = ora.loss_grad(prob, d, w, po, want_grad=False)
    return lo[2]


def test_adam_200_final_loss_spread_under_fp32_sized_gradient_errors():
    prob = synth.make_deconv(1)
    rng = np.random.default_rng(5)
    d, w = synth.add_noise(ora.forward_model(prob, prob.params_true), rng)
    p0 = synth.eval_point(prob, "init", rng)
    ref = _adam_run(prob, d, w, p0, None)
    spread = max(abs(_adam_run(prob, d, w, p0, s) - ref) / abs(ref) for s in (0, 1))
    assert spread > 1e-4
    assert spread < ADAM200_LOSS_BAR / 2
