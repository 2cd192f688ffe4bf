"""Whole-evaluation parity at full size: the supernova workload (1000 ragged
epochs, 256^2 grid) and the large field (12 epochs of 256^2 data, 512^2 grid, 30
sources, 8 scales), loss and every gradient block against the FP64 oracle at
three points: "init" (P0), "near" (P1) and the oracle's own Adam state after 50
steps from P0 (P2, tests/golden/p2_cfg<k>.npz, written by tests/golden/make_p2.py
from the oracle alone). Plans: the FFT algorithm, the autotuned plan, and the
direct algorithm.

Bars as everywhere: loss relative error <= 1e-6, gradient relative error <= 1e-4
per block and overall, after the tie rule for zero starlet coefficients.
The oracle's part runs on the host's cores (about a minute per supernova point on
16 threads).
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as ora
from oracle import parity
from paper_2402_08725_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_p2  # noqa: E402  (the data recipe P2 was made on)

_DATA = {}
_ORA = {}
_PLANS = {}


def _say(msg):
    print(msg, flush=True)


def _setup(cfg):
    """Problem, data and weights of the full-size workload, and its three points."""
    if cfg not in _DATA:
        _say(f"cfg{cfg}: oracle forward model for the data")
        prob, d, w, rng = make_p2.full_size_data(cfg)
        pts = {"P0": synth.eval_point(prob, "init", rng)}
        pts["P1"] = synth.eval_point(prob, "near", np.random.default_rng(make_p2.DATA_SEED + 1))
        _DATA[cfg] = (prob, d, w, pts)
    return _DATA[cfg]


def _point(cfg, point):
    prob, _, _, pts = _setup(cfg)
    if point not in pts:  # P2, stored by the generator script
        with np.load(os.path.join(HERE, "golden", f"p2_cfg{cfg}.npz")) as z:
            pts[point] = z["x"].astype(np.float64)
        assert pts[point].size == prob.n_params
    return pts[point]


def _plan(cfg, kind):
    st = pytest.importorskip("paper_2402_08725_amd.starred")
    key = (cfg, kind)
    if key not in _PLANS:
        prob, d, w, _ = _setup(cfg)
        algo = {"fft": st.CONV_FFT, "auto": st.CONV_AUTO, "direct": st.CONV_DIRECT}[kind]
        plan = st.Plan.for_problem(prob, conv_algo=algo)
        plan.set_frames(d, w, prob.kernels, prob.W)
        _say(f"cfg{cfg} {kind} plan: " + ", ".join(
            f"n{c['n']}:{'dir' if c['algo'] == 1 else ('fused' if c['fused'] else 'lines')}" for c in plan.classes()))
        _PLANS[key] = plan
    return _PLANS[key]


def _oracle(cfg, point, alpha_dev):
    key = (cfg, point)
    if key not in _ORA:
        prob, d, w, _ = _setup(cfg)
        p = _point(cfg, point)
        NN = prob.N * prob.N
        so, nsub = parity.tie_override(prob.N, prob.J, p[:NN], alpha_dev)
        _say(f"cfg{cfg} {point}: oracle loss and gradient ({nsub} tied coefficients)")
        _ORA[key] = ora.loss_grad(prob, d, w, p, sgn_override=so)
    return _ORA[key]


CASES = [(4, "fft"), (4, "auto"), (4, "direct"), (5, "fft"), (5, "auto"), (5, "direct")]


@pytest.mark.parametrize("point", ["P0", "P1", "P2"])
@pytest.mark.parametrize("cfg,kind", CASES, ids=[f"cfg{c}-{k}" for c, k in CASES])
def test_full_size_loss_and_gradient(cfg, kind, point):
    prob, d, w, _ = _setup(cfg)
    plan = _plan(cfg, kind)
    p = _point(cfg, point)
    NN = prob.N * prob.N
    loss, grad = plan.loss_grad(p)
    alpha_dev = plan.starlet_fwd(p[:NN]).cpu().numpy()
    loss = loss.cpu().numpy()
    grad = grad.cpu().numpy().astype(np.float64)
    lo, go = _oracle(cfg, point, alpha_dev)
    rl = abs(loss[2] - lo[2]) / abs(lo[2])
    blocks = {k: parity.rel_err(parity.deconv_blocks(prob, grad)[k], v)
              for k, v in parity.deconv_blocks(prob, go).items() if np.linalg.norm(v) > 0}
    rg = parity.rel_err(grad, go)
    _say(f"cfg{cfg} {kind} {point}: loss {loss[2]:.9e} oracle {lo[2]:.9e} rel {rl:.2e}; "
         f"grad rel {rg:.2e} {', '.join(f'{k} {v:.2e}' for k, v in blocks.items())}")
    assert rl <= 1e-6
    assert rg <= 1e-4
    for k, v in blocks.items():
        assert v <= 1e-4, (k, v)
