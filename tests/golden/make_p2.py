"""Writes the third parity point P2 of the full-size workloads: the oracle's own
Adam state after 50 steps from the "init" point, on the same seeded data the GPU
parity tests build (oracle forward model at the truth plus noise).

Calls only the FP64 oracle and the input generators; the HIP library is not
involved. Usage: python tests/golden/make_p2.py [cfg ...] (default 5 4).
Output: tests/golden/p2_cfg<cfg>.npz with the FP32 parameter vector `x` and the
oracle's loss there (`loss`, for reference).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as ora  # noqa: E402
from paper_2402_08725_amd import synth  # noqa: E402

# data seed of the full-size whole-evaluation tests, and the Adam run
DATA_SEED = 21
ADAM_STEPS = 50


def full_size_data(cfg):
    """The problem, data, weights and the rng state after them (the test recipe)."""
    prob = synth.make_deconv(cfg)
    rng = np.random.default_rng(DATA_SEED)
    d, w = synth.add_noise(ora.forward_model(prob, prob.params_true), rng)
    return prob, d, w, rng


def make(cfg):
    prob, d, w, rng = full_size_data(cfg)
    p = synth.eval_point(prob, "init", rng)
    lr = prob.lr_vector()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    t0 = time.time()
    for t in range(1, ADAM_STEPS + 1):
        loss, g = ora.loss_grad(prob, d, w, p)
        ora.adam_step(p, g, m, v, t, lr)
        print(f"cfg{cfg} step {t}: loss {loss[2]:.9e} ({time.time() - t0:.0f} s)", flush=True)
    x = p.astype(np.float32)
    lo, _ = ora.loss_grad(prob, d, w, x.astype(np.float64), want_grad=False)
    np.savez_compressed(os.path.join(HERE, f"p2_cfg{cfg}.npz"), x=x, loss=lo, steps=ADAM_STEPS,
                        data_seed=DATA_SEED)
    print(f"cfg{cfg}: P2 written, loss {lo[2]:.9e}", flush=True)


if __name__ == "__main__":
    for c in (sys.argv[1:] or ["5", "4"]):
        make(int(c))
