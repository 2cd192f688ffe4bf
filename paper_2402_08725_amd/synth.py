"""Seeded synthetic inputs with the shapes of the paper's workloads.

This module only draws inputs: truth scenes (Sersic hosts, point-source positions
and light curves), per-epoch narrow-PSF kernels, noise, and per-scale starlet
weights. It holds none of the method's arithmetic (no rendering of the model,
no convolution, no subsampling, no starlet transform); the noiseless model image
that the noise is added to is computed by the caller.

Workloads (all values rounded to FP32 so that the FP32 device path and the FP64
oracle see identical inputs):

  cfg1  4 epochs of 32x32 data, s=2 (64x64 grid), 64x64 Moffat kernels, 1 point
        source, round Sersic n=1 host, J=3, lambda=3   (runtime study, Sec. 2.4)
  cfg2  100 epochs of 64x64, s=2 (128x128), 128x128 kernels, 4 point sources with
        log-normal 0.3 dex amplitudes, Sersic n=2 q=0.4 arc host, J=6
        (lensed-quasar light curves, Sec. 4.2)
  cfg3  PSF mode: 30 star stamps of 64x64 at s=3 (192x192 PSF grid), elliptical
        Moffat plus a residual pixel grid, J=5   (PSF reconstruction, Sec. 3)
  cfg4  1000 epochs, ragged stamp sides {32,48,64,96,128}, s=2, 256x256 host grid,
        one transient (rise then exponential decay), J=6   (supernova, Sec. 4.1)
  cfg5  12 epochs of 256x256, s=2 (512x512), 128x128 kernels (Moffat + 10 %
        Gaussian halo), 30 point sources over 5 Sersic galaxies, J=8
        (crowded JWST-like field, Sec. 4.3)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Std of each starlet plane for unit white noise (B3 a-trous), used to give the
# per-scale weights a realistic shape.
_STARLET_NOISE = [0.8907, 0.2007, 0.0856, 0.0413, 0.0205, 0.0103, 0.0052, 0.0026,
                  0.0013, 0.00065, 0.00033, 0.00016]

FWHM_R = 2.0  # FWHM of the target Gaussian r in fine pixels (Sec. 2.1)


def f32(a):
    """Round to FP32 and return float64 holding FP32-representable values."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rng_for(cfg: int, rep: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * cfg + rep))


# --------------------------------------------------------------------------- #
# Profiles used to draw truth scenes and kernels                               #
# --------------------------------------------------------------------------- #

def sersic_bn(n: float) -> float:
    """Ciotti & Bertin (1999) asymptotic series for b_n."""
    return (2 * n - 1.0 / 3 + 4.0 / (405 * n) + 46.0 / (25515 * n * n)
            + 131.0 / (1148175 * n ** 3) - 2194697.0 / (30690717750 * n ** 4))


def sersic_image(N: int, xc: float, yc: float, flux: float, n: float, r_e: float,
                 q: float = 1.0, phi: float = 0.0, sub: int = 4) -> np.ndarray:
    """Elliptical Sersic profile point-sampled at pixel centres, with sub x sub
    sampling inside 2 px of the centre, scaled so the grid sum equals flux."""
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    bn = sersic_bn(n)

    def prof(xx, yy):
        dx, dy = xx - xc, yy - yc
        u = math.cos(phi) * dx + math.sin(phi) * dy
        v = -math.sin(phi) * dx + math.cos(phi) * dy
        R = np.sqrt(u * u + (v / q) ** 2)
        return np.exp(-bn * ((R / r_e) ** (1.0 / n) - 1.0))

    img = prof(x, y)
    near = np.hypot(x - xc, y - yc) < 2.0
    if near.any():
        offs = (np.arange(sub) + 0.5) / sub - 0.5
        acc = np.zeros(int(near.sum()))
        for oy in offs:
            for ox in offs:
                acc += prof(x[near] + ox, y[near] + oy)
        img[near] = acc / (sub * sub)
    return img * (flux / img.sum())


def moffat_alpha(fwhm: float, beta: float) -> float:
    return fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))


def moffat_kernel(K: int, fwhm: float, beta: float, halo_frac: float = 0.0,
                  halo_fwhm: float = 0.0) -> np.ndarray:
    """Round Moffat (optionally plus a Gaussian halo) centred at floor(K/2),
    normalised to unit sum: a per-epoch narrow PSF s_i."""
    c = K // 2
    y, x = np.mgrid[0:K, 0:K].astype(np.float64)
    r2 = (x - c) ** 2 + (y - c) ** 2
    al = moffat_alpha(fwhm, beta)
    m = (1.0 + r2 / al ** 2) ** (-beta)
    m /= m.sum()
    if halo_frac > 0:
        sg = halo_fwhm / (2 * math.sqrt(2 * math.log(2)))
        g = np.exp(-r2 / (2 * sg * sg))
        g /= g.sum()
        m = (1 - halo_frac) * m + halo_frac * g
    return m


# --------------------------------------------------------------------------- #
# Deconvolution problems                                                       #
# --------------------------------------------------------------------------- #

@dataclass
class DeconvProblem:
    name: str
    E: int
    n: np.ndarray          # int32 [E] data side per frame
    K: np.ndarray          # int32 [E] kernel side per frame
    s: int
    N: int
    M: int
    J: int
    lam: float
    kernels: np.ndarray    # packed K_i^2, float64 holding FP32 values
    h: np.ndarray          # truth h (N^2)
    Gamma: np.ndarray      # truth Gamma (E)
    a: np.ndarray          # truth a (E*M, epoch-major)
    c: np.ndarray          # truth c (M*2: cx, cy)
    W: np.ndarray          # per-scale weights [J]
    w_stride: int = 0
    fwhm: float = FWHM_R
    sigma_bg: float = 10.0
    adam_lr: dict = field(default_factory=dict)

    @property
    def n_params(self) -> int:
        return self.N * self.N + self.E + self.E * self.M + 2 * self.M

    def pack(self, h=None, Gamma=None, a=None, c=None) -> np.ndarray:
        return f32(np.concatenate([
            np.ravel(self.h if h is None else h), np.ravel(self.Gamma if Gamma is None else Gamma),
            np.ravel(self.a if a is None else a), np.ravel(self.c if c is None else c)]))

    def unpack(self, p):
        NN = self.N * self.N
        E, M = self.E, self.M
        return (p[:NN], p[NN:NN + E], p[NN + E:NN + E + E * M], p[NN + E + E * M:])

    @property
    def params_true(self) -> np.ndarray:
        return self.pack()

    @property
    def data_size(self) -> int:
        return int(np.sum(self.n.astype(np.int64) ** 2))

    @property
    def fine_size(self) -> int:
        return int(np.sum((self.s * self.n.astype(np.int64)) ** 2))

    def lr_vector(self) -> np.ndarray:
        NN = self.N * self.N
        lr = np.empty(self.n_params)
        lr[:NN] = self.adam_lr.get("h", 0.5)
        lr[NN:NN + self.E] = self.adam_lr.get("Gamma", 0.05)
        lr[NN + self.E:NN + self.E + self.E * self.M] = self.adam_lr.get("a", 20.0)
        lr[NN + self.E + self.E * self.M:] = self.adam_lr.get("c", 0.01)
        return lr


def starlet_weights(J: int, sigma_h: float) -> np.ndarray:
    """Per-scale weights with the starlet's white-noise shape, scaled to a
    propagated-noise level sigma_h; the coarse plane is not penalised."""
    W = np.array([_STARLET_NOISE[j] if j < len(_STARLET_NOISE) else 0.0 for j in range(J)])
    W = W * sigma_h
    W[J - 1] = 0.0
    return f32(W)


def _sigma_h(kernels_list, s, w_level) -> float:
    # Std of the back-propagated white noise of every epoch summed on the fine grid.
    tot = 0.0
    for k in kernels_list:
        tot += w_level * s * s * float(np.sum(k * k))
    return math.sqrt(tot)


def make_deconv(cfg: int, rep: int = 0, E: int | None = None, sizes=None,
                N: int | None = None) -> DeconvProblem:
    """Draw the truth and kernels of deconvolution workload `cfg` (1, 2, 4 or 5).

    E overrides the number of epochs (a smaller instance with the same shapes);
    sizes overrides the ragged side choices of cfg4; N overrides its host grid."""
    rng = rng_for(cfg, rep)
    s = 2
    if cfg == 1:
        E = E or 4
        n = np.full(E, 32, np.int32)
        N = 64
        K = np.full(E, 64, np.int32)
        fwhm = rng.uniform(3, 5, E)
        kernels = [moffat_kernel(64, fw, 2.5) for fw in fwhm]
        M, J, lam = 1, 3, 3.0
        ctr = (N - 1) / 2.0
        c = np.array([ctr + s * rng.uniform(-0.5, 0.5), ctr + s * rng.uniform(-0.5, 0.5)])
        a = np.full((E, M), 1e4)
        h = sersic_image(N, ctr, ctr, 5e3, 1.0, 4.0)
        adam_lr = {"h": 0.5, "Gamma": 0.05, "a": 20.0, "c": 0.01}
    elif cfg == 2:
        E = E or 100
        n = np.full(E, 64, np.int32)
        N = 128
        K = np.full(E, 128, np.int32)
        fwhm = rng.uniform(3, 8, E)
        kernels = [moffat_kernel(128, fw, 2.5) for fw in fwhm]
        M, J, lam = 4, 6, 3.0
        ctr = (N - 1) / 2.0
        rad = 6.0
        c = np.array([ctr + rad, ctr, ctr, ctr + rad, ctr - rad, ctr, ctr, ctr - rad])
        c = c + rng.uniform(-0.5, 0.5, 8)
        base = np.array([5e3, 3e3, 2e3, 1e3])
        a = base[None, :] * 10 ** (0.3 * rng.standard_normal((E, M)))
        h = sersic_image(N, ctr, ctr, 2e4, 2.0, 10.0, q=0.4, phi=0.6)
        adam_lr = {"h": 0.5, "Gamma": 0.05, "a": 20.0, "c": 0.01}
    elif cfg == 4:
        E = E or 1000
        choices = np.array(sizes if sizes is not None else [32, 48, 64, 96, 128], np.int32)
        n = rng.choice(choices, E).astype(np.int32)
        N = N or 2 * int(choices.max())
        K = np.minimum(2 * n, 128).astype(np.int32)
        fwhm = rng.uniform(2.5, 9, E)
        kernels = [moffat_kernel(int(k), fw, 2.5) for k, fw in zip(K, fwhm)]
        M, J, lam = 1, min(6, int(math.floor(math.log2(max(2, 2 * int(choices.min()) - 1)))) + 1), 3.0
        ctr = (N - 1) / 2.0
        c = np.array([ctr + 8.0, ctr])
        t0 = int(0.6 * E)
        idx = np.arange(E)
        xx = (idx - t0) / (15.0 * E / 1000.0)
        a = np.where(idx < t0, 0.0, 2e4 * xx * np.exp(1 - xx))[:, None]
        h = sersic_image(N, ctr, ctr, 5e4, 1.0, 12.0, q=0.6, phi=0.3)
        adam_lr = {"h": 0.5, "Gamma": 0.05, "a": 20.0, "c": 0.01}
    elif cfg == 5:
        E = E or 12
        nside = 256
        n = np.full(E, nside, np.int32)
        N = 2 * nside
        K = np.full(E, 128, np.int32)
        fwhm = rng.uniform(3, 8, E)
        kernels = [moffat_kernel(128, fw, 2.5, 0.1, 4 * fw) for fw in fwhm]
        M, J, lam = 30, 8, 3.0
        c = rng.uniform(8, N - 9, 2 * M)
        a = 10 ** rng.uniform(2, 5, M)[None, :] * np.exp(0.1 * rng.standard_normal((E, M)))
        h = np.zeros((N, N))
        for _ in range(5):
            h += sersic_image(N, rng.uniform(N / 4, 3 * N / 4), rng.uniform(N / 4, 3 * N / 4),
                              10 ** rng.uniform(4, 6), rng.uniform(0.5, 4), rng.uniform(5, 40),
                              q=rng.uniform(0.3, 1), phi=rng.uniform(0, math.pi))
        adam_lr = {"h": 0.5, "Gamma": 0.05, "a": 20.0, "c": 0.01}
    else:
        raise ValueError(f"no deconvolution workload {cfg}")

    kern = f32(np.concatenate([np.ravel(k) for k in kernels]))
    w_level = 1.0 / (10.0 ** 2)
    W = starlet_weights(J, _sigma_h(kernels, s, w_level))
    return DeconvProblem(
        name=f"cfg{cfg}", E=E, n=n, K=K.astype(np.int32), s=s, N=N, M=M, J=J, lam=lam,
        kernels=kern, h=f32(h).ravel(), Gamma=f32(np.zeros(E)), a=f32(np.asarray(a)).ravel(),
        c=f32(c).ravel(), W=W, adam_lr=adam_lr)


def subset(prob: DeconvProblem, frames) -> DeconvProblem:
    """The same workload restricted to some of its frames (inputs sliced, nothing
    computed): kernels, Gamma and a of those frames; h, c and W unchanged."""
    idx = np.asarray(frames, dtype=np.int64)
    koff = np.concatenate([[0], np.cumsum(prob.K.astype(np.int64) ** 2)])
    kern = np.concatenate([prob.kernels[koff[i]:koff[i + 1]] for i in idx])
    a = prob.a.reshape(prob.E, prob.M)[idx].ravel()
    return DeconvProblem(
        name=f"{prob.name}[{len(idx)} frames]", E=len(idx), n=prob.n[idx].copy(), K=prob.K[idx].copy(),
        s=prob.s, N=prob.N, M=prob.M, J=prob.J, lam=prob.lam, kernels=kern, h=prob.h, Gamma=prob.Gamma[idx].copy(),
        a=a, c=prob.c, W=prob.W, w_stride=prob.w_stride, fwhm=prob.fwhm, sigma_bg=prob.sigma_bg,
        adam_lr=dict(prob.adam_lr))


def subset_params(prob: DeconvProblem, params: np.ndarray, frames) -> np.ndarray:
    """A parameter vector of prob restricted to some frames (see subset)."""
    idx = np.asarray(frames, dtype=np.int64)
    h, G, a, c = prob.unpack(np.asarray(params))
    return np.concatenate([h, G[idx], a.reshape(prob.E, prob.M)[idx].ravel(), c])


def make_small_deconv(seed: int, E: int, sides, K, s: int, N: int, M: int, J: int,
                      lam: float = 3.0, w_stride: int = 0) -> DeconvProblem:
    """A small random deconvolution instance for property and parity tests:
    arbitrary ragged sides, arbitrary (odd or even) kernel sides, any s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.array([sides[i % len(sides)] for i in range(E)], np.int32)
    Ks = np.array([K[i % len(K)] for i in range(E)] if np.ndim(K) else [K] * E, np.int32)
    kernels = [moffat_kernel(int(k), rng.uniform(1.5, 4), 2.5) for k in Ks]
    ctr = (N - 1) / 2.0
    c = rng.uniform(ctr - N / 4, ctr + N / 4, 2 * M)
    a = 10 ** rng.uniform(2, 4, (E, M))
    h = sersic_image(N, ctr + 1.3, ctr - 0.7, 3e3, 1.5, N / 8, q=0.7, phi=0.4)
    h += rng.normal(0, 5.0, (N, N))
    Gam = rng.normal(0, 3.0, E)
    if w_stride:
        W = f32(rng.uniform(0.5, 2.0, (J, N, N)) * 3.0).ravel()
    else:
        W = starlet_weights(J, _sigma_h(kernels, s, 0.01))
    return DeconvProblem(
        name=f"small{seed}", E=E, n=n, K=Ks, s=s, N=N, M=M, J=J, lam=lam,
        kernels=f32(np.concatenate([np.ravel(k) for k in kernels])), h=f32(h).ravel(),
        Gamma=f32(Gam), a=f32(a).ravel(), c=f32(c), W=W, w_stride=w_stride)


def add_noise(model: np.ndarray, rng: np.random.Generator, sigma_bg: float = 10.0,
              poisson: bool = True):
    """Data and inverse variance from a noiseless model image: Gaussian background
    of std sigma_bg plus Poisson noise of the (positive) model, gain 1."""
    pos = np.maximum(model, 0.0)
    d = model + rng.normal(0.0, sigma_bg, model.shape)
    if poisson:
        d = d + (rng.poisson(pos) - pos)
    w = 1.0 / (sigma_bg ** 2 + (pos if poisson else np.zeros_like(pos)))
    return f32(d), f32(w)


def eval_point(prob: DeconvProblem, which: str, rng: np.random.Generator) -> np.ndarray:
    """Parameter vectors at which loss and gradient are compared.
    'init': h = 0, Gamma = 0, a perturbed by U(0.5,1.5), c by U(-1,1) fine px.
    'near': truth plus small perturbations of every block."""
    if which == "init":
        return prob.pack(h=np.zeros(prob.N * prob.N), Gamma=np.zeros(prob.E),
                         a=prob.a * rng.uniform(0.5, 1.5, prob.a.shape),
                         c=prob.c + rng.uniform(-1, 1, prob.c.shape))
    if which == "near":
        hmax = max(float(np.abs(prob.h).max()), 1.0)
        return prob.pack(h=prob.h + 0.05 * hmax * rng.standard_normal(prob.h.shape),
                         Gamma=prob.Gamma + rng.normal(0, prob.sigma_bg / prob.s ** 2, prob.E),
                         a=prob.a * np.exp(0.1 * rng.standard_normal(prob.a.shape)),
                         c=prob.c + 0.25 * rng.standard_normal(prob.c.shape))
    raise ValueError(which)


# --------------------------------------------------------------------------- #
# PSF-reconstruction problems                                                  #
# --------------------------------------------------------------------------- #

@dataclass
class PSFProblem:
    name: str
    S: int
    n: int
    s: int
    N: int
    J: int
    lam: float
    eta: np.ndarray        # (A, alpha_x, alpha_y, phi, beta)
    b: np.ndarray          # N^2 residual grid
    a: np.ndarray          # S amplitudes
    c: np.ndarray          # S*2 centre offsets (fine px)
    W: np.ndarray
    w_stride: int = 0
    fwhm: float = FWHM_R
    sigma_bg: float = 10.0

    @property
    def n_params(self) -> int:
        return 5 + self.N * self.N + 3 * self.S

    def pack(self, eta=None, b=None, a=None, c=None) -> np.ndarray:
        return f32(np.concatenate([
            np.ravel(self.eta if eta is None else eta), np.ravel(self.b if b is None else b),
            np.ravel(self.a if a is None else a), np.ravel(self.c if c is None else c)]))

    @property
    def params_true(self) -> np.ndarray:
        return self.pack()

    @property
    def data_size(self) -> int:
        return self.S * self.n * self.n


def make_psf(cfg: int = 3, rep: int = 0, S: int | None = None, n: int | None = None,
             s: int | None = None, J: int | None = None) -> PSFProblem:
    """PSF-mode workload: S star stamps of n x n at subsampling s."""
    rng = rng_for(cfg, rep)
    S = S or 30
    n = n or 64
    s = s or 3
    N = n * s
    J = J or 5
    beta = rng.uniform(2, 4)
    q = rng.uniform(0.7, 1.0)
    phi = rng.uniform(0, math.pi)
    fw = rng.uniform(9, 15) * N / 192.0
    ax = moffat_alpha(fw, beta)
    ay = ax * q
    c0 = N // 2
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    dx, dy = x - c0, y - c0
    u = math.cos(phi) * dx + math.sin(phi) * dy
    v = -math.sin(phi) * dx + math.cos(phi) * dy
    prof = (1 + (u / ax) ** 2 + (v / ay) ** 2) ** (-beta)
    A = 0.95 / prof.sum()
    rr = np.hypot(dx, dy)
    ann = np.exp(-0.5 * ((rr - 2 * fw) / (0.5 * fw)) ** 2)
    b = 0.05 * ann / ann.sum()
    a = 10 ** rng.uniform(3, 6, S)
    c = rng.uniform(-1.5, 1.5, 2 * S)
    W = starlet_weights(J, 10.0 * math.sqrt(S) * 0.05)
    return PSFProblem(name=f"psf{cfg}", S=S, n=n, s=s, N=N, J=J, lam=3.0,
                      eta=f32([A, ax, ay, phi, beta]), b=f32(b).ravel(), a=f32(a), c=f32(c), W=W)


def psf_eval_point(prob: PSFProblem, which: str, rng: np.random.Generator) -> np.ndarray:
    if which == "init":
        eta = prob.eta.copy()
        eta[1:3] *= rng.uniform(0.8, 1.2, 2)
        eta[4] *= rng.uniform(0.9, 1.1)
        return prob.pack(eta=eta, b=np.zeros_like(prob.b),
                         a=prob.a * rng.uniform(0.5, 1.5, prob.S),
                         c=prob.c + rng.uniform(-1, 1, 2 * prob.S))
    if which == "near":
        eta = prob.eta * (1 + 0.02 * rng.standard_normal(5))
        bmax = float(np.abs(prob.b).max())
        return prob.pack(eta=eta, b=prob.b + 0.1 * bmax * rng.standard_normal(prob.b.shape),
                         a=prob.a * np.exp(0.05 * rng.standard_normal(prob.S)),
                         c=prob.c + 0.2 * rng.standard_normal(2 * prob.S))
    raise ValueError(which)
