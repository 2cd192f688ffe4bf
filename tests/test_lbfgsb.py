"""The host L-BFGS-B iteration of the library (generalized Cauchy point, subspace
minimisation, Moré-Thuente line search) against scipy's L-BFGS-B, iterate by
iterate, on analytic problems and on the FP64 oracle's losses. Both sides are FP64
and follow the same published algorithm, so the iterates agree to rounding (the
bars below leave room for its slow growth). CPU only."""
import numpy as np
import pytest
from scipy.optimize import minimize, rosen, rosen_der

from oracle import oracle as ora
from paper_2402_08725_amd import synth


def _st():
    from paper_2402_08725_amd import build, starred
    import os
    if not os.path.exists(starred.LIB_PATH):
        build.build()
    return starred


def _both(fun, x0, lo, hi, iters, m=10, factr=1e7, pgtol=1e-5):
    st = _st()
    xs_s = []
    bounds = None if lo is None else list(zip(lo, hi))
    minimize(fun, x0, jac=True, method="L-BFGS-B", bounds=bounds,
             options=dict(maxiter=iters, maxcor=m, ftol=factr * np.finfo(float).eps, gtol=pgtol),
             callback=lambda xk: xs_s.append(np.array(xk, dtype=np.float64)))
    xs_m = []
    opt = st.LBFGSB(len(x0), m=m, lo=lo, hi=hi, factr=factr, pgtol=pgtol)
    opt.minimize(fun, x0, iters, callback=lambda xk: xs_m.append(xk))
    return xs_s, xs_m


def _compare(xs_s, xs_m, k, rtol):
    assert len(xs_m) >= k and len(xs_s) >= k, (len(xs_s), len(xs_m))
    for i in range(k):
        scale = max(np.abs(xs_s[i]).max(), 1.0)
        err = np.abs(xs_s[i] - xs_m[i]).max() / scale
        assert err <= rtol, (i, err)


@pytest.mark.parametrize("bounds", ["none", "box", "partial"])
def test_lbfgsb_rosenbrock_iterates_match_scipy(bounds):
    n = 10
    x0 = np.full(n, -1.2)
    x0[1::2] = 1.0
    lo = hi = None
    if bounds == "box":
        lo, hi = np.full(n, -2.0), np.full(n, 0.8)
    elif bounds == "partial":
        lo, hi = np.full(n, -np.inf), np.full(n, np.inf)
        lo[::3] = -0.5
        hi[1::4] = 0.5
    xs_s, xs_m = _both(lambda x: (rosen(x), rosen_der(x)), x0, lo, hi, 25)
    _compare(xs_s, xs_m, 25, 1e-9)


def test_lbfgsb_bounded_quadratic_reaches_the_kkt_point():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 20))
    Q = A.T @ A + 0.1 * np.eye(20)
    b = rng.standard_normal(20)
    lo, hi = np.full(20, -0.3), np.full(20, 0.3)
    xs_s, xs_m = _both(lambda x: (0.5 * x @ Q @ x - b @ x, Q @ x - b), np.zeros(20), lo, hi, 200, factr=10.0,
                       pgtol=1e-9)
    _compare(xs_s, xs_m, min(len(xs_s), 15), 1e-10)
    x = xs_m[-1]
    g = Q @ x - b
    # projected gradient vanishes: interior entries have g = 0, entries at a bound push outward
    pg = np.where(x <= lo + 1e-12, np.minimum(g, 0.0), np.where(x >= hi - 1e-12, np.maximum(g, 0.0), g))
    assert np.abs(pg).max() <= 1e-6


def test_lbfgsb_on_the_oracle_deconvolution_loss():
    """A small joint deconvolution (Eqs. 9-11) with h >= 0 and a_ik >= 0: the
    library's iterates against scipy's on the oracle's loss and gradient."""
    prob = synth.make_small_deconv(seed=81, E=3, sides=[12, 16, 10], K=[7, 9, 5], s=2, N=40, M=2, J=3)
    rng = np.random.default_rng(81)
    d, w = synth.add_noise(ora.forward_model(prob, prob.params_true), rng)
    p0 = synth.eval_point(prob, "init", rng)
    NN, E, M = prob.N ** 2, prob.E, prob.M
    lo = np.full(prob.n_params, -np.inf)
    hi = np.full(prob.n_params, np.inf)
    lo[:NN] = 0.0
    lo[NN + E:NN + E + E * M] = 0.0

    def fun(x):
        loss, g = ora.loss_grad(prob, d, w, x)
        return loss[2], g
    xs_s, xs_m = _both(fun, np.maximum(p0, lo), lo, hi, 12)
    _compare(xs_s, xs_m, 12, 1e-7)


def test_lbfgsb_on_the_oracle_psf_loss():
    """PSF mode (Eqs. 2-7) with positive Moffat widths and exponent and positive
    amplitudes: the iterates against scipy's on the oracle's loss."""
    prob = synth.make_psf(3, S=4, n=16, s=3, J=4)
    rng = np.random.default_rng(82)
    m = ora.psf_model(prob, prob.params_true)
    d, w = synth.add_noise(m, rng, poisson=False)
    p0 = synth.psf_eval_point(prob, "init", rng)
    NN, S = prob.N ** 2, prob.S
    lo = np.full(prob.n_params, -np.inf)
    hi = np.full(prob.n_params, np.inf)
    lo[1:3] = 0.5
    lo[4] = 1.0
    lo[5 + NN:5 + NN + S] = 0.0

    def fun(x):
        loss, g = ora.psf_loss_grad(prob, d, w, x)
        return loss[2], g
    xs_s, xs_m = _both(fun, np.maximum(p0, lo), lo, hi, 10)
    _compare(xs_s, xs_m, 10, 1e-7)
