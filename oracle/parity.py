"""Comparison helpers between a device result and the oracle (test infrastructure).

The L1 prior is not differentiable where a starlet coefficient is 0: any value of
lambda W in [-1, 1] is a valid subgradient there, and an FP32 device and the
FP64 oracle may legitimately disagree on the sign of a coefficient that is zero
up to rounding. For coefficients with |alpha| <= 2^-17 * max |alpha_j| the
comparison takes the sign the device itself computed (from its own starlet
transform) and substitutes it into the oracle's subgradient.
"""
from __future__ import annotations

import numpy as np

from . import oracle as ora

TIE_REL = 2.0 ** -17


def tie_override(N, J, img_params, alpha_dev):
    """int8 override array for the oracle and the number of substituted signs."""
    alpha = ora.starlet_fwd(N, J, img_params).reshape(J, -1)
    ad = np.asarray(alpha_dev, dtype=np.float64).reshape(J, -1)
    so = np.full(alpha.shape, 2, np.int8)
    nsub = 0
    for j in range(J):
        tau = TIE_REL * max(np.abs(alpha[j]).max(), 1e-300)
        tie = np.abs(alpha[j]) <= tau
        so[j, tie] = np.sign(ad[j, tie]).astype(np.int8)
        nsub += int(tie.sum())
    return so.ravel(), nsub


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def deconv_blocks(prob, g):
    NN = prob.N * prob.N
    E, M = prob.E, prob.M
    return {"h": g[:NN], "Gamma": g[NN:NN + E], "a": g[NN + E:NN + E + E * M],
            "c": g[NN + E + E * M:]}


def psf_blocks(prob, g):
    NN = prob.N * prob.N
    return {"eta": g[:5], "b": g[5:5 + NN], "a": g[5 + NN:5 + NN + prob.S],
            "c": g[5 + NN + prob.S:]}
