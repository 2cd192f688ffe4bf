"""ctypes wrapper of the FP64 oracle (starred_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "starred_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_B = ctypes.POINTER(ctypes.c_byte)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (portable x86-64-v3 code, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        v = ctypes.c_void_p
        _lib.ora_sigma_from_fwhm.restype = ctypes.c_double
        _lib.ora_sigma_from_fwhm.argtypes = [ctypes.c_double]
        for name in ["ora_render_scene", "ora_conv_sub", "ora_conv_sub_adj", "ora_starlet_fwd",
                     "ora_starlet_adj", "ora_loss_grad", "ora_forward_model", "ora_moffat",
                     "ora_psf_render", "ora_psf_model", "ora_psf_loss_grad", "ora_adam_step",
                     "ora_noise_variance", "ora_noise_weights_mc", "ora_pts_term", "ora_adabelief_step",
                     "ora_lbfgs_direction", "ora_set_num_threads", "ora_render_scene_xf",
                     "ora_loss_grad_xf"]:
            getattr(_lib, name).restype = None
        _lib.ora_philox4x32_10.restype = None
        _lib.ora_lambda_pts_estimate.restype = ctypes.c_double
        _lib.ora_normal.restype = ctypes.c_double
        _lib.ora_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        _lib.ora_num_threads.restype = ctypes.c_int
        _lib.ora_frame_offsets.restype = ctypes.c_int
        del v
    return _lib


def _d(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().ora_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's frame loops (n <= 0: every processor)."""
    lib().ora_set_num_threads(int(n))


def sigma_from_fwhm(fwhm: float) -> float:
    return lib().ora_sigma_from_fwhm(fwhm)


def frame_offsets(n, s, N):
    n = _i32(n)
    o = np.zeros(len(n), np.int32)
    rc = lib().ora_frame_offsets(len(n), n.ctypes.data_as(_I), s, N, o.ctypes.data_as(_I))
    if rc != 0:
        raise ValueError("frame does not fit the grid")
    return o


def render_scene(n, s, N, M, fwhm, params):
    n = _i32(n)
    params = _f64(params)
    out = np.zeros(int(np.sum((s * n.astype(np.int64)) ** 2)))
    lib().ora_render_scene(len(n), n.ctypes.data_as(_I), s, N, M, ctypes.c_double(fwhm),
                           _d(params), _d(out))
    return out


def conv_sub(n, K, s, kernels, scene):
    n, K = _i32(n), _i32(K)
    kernels, scene = _f64(kernels), _f64(scene)
    out = np.zeros(int(np.sum(n.astype(np.int64) ** 2)))
    lib().ora_conv_sub(len(n), n.ctypes.data_as(_I), K.ctypes.data_as(_I), s, _d(kernels),
                       _d(scene), _d(out))
    return out


def conv_sub_adj(n, K, s, kernels, resid):
    n, K = _i32(n), _i32(K)
    kernels, resid = _f64(kernels), _f64(resid)
    out = np.zeros(int(np.sum((s * n.astype(np.int64)) ** 2)))
    lib().ora_conv_sub_adj(len(n), n.ctypes.data_as(_I), K.ctypes.data_as(_I), s, _d(kernels),
                           _d(resid), _d(out))
    return out


def starlet_fwd(N, J, img):
    img = _f64(img)
    out = np.zeros(J * N * N)
    lib().ora_starlet_fwd(N, J, _d(img), _d(out))
    return out


def starlet_adj(N, J, coeffs):
    coeffs = _f64(coeffs)
    out = np.zeros(N * N)
    lib().ora_starlet_adj(N, J, _d(coeffs), _d(out))
    return out


def forward_model(prob, params):
    frame_offsets(prob.n, prob.s, prob.N)
    n, K = _i32(prob.n), _i32(prob.K)
    params, kernels = _f64(params), _f64(prob.kernels)
    out = np.zeros(int(np.sum(n.astype(np.int64) ** 2)))
    lib().ora_forward_model(prob.E, n.ctypes.data_as(_I), K.ctypes.data_as(_I), prob.s, prob.N,
                            prob.M, ctypes.c_double(prob.fwhm), _d(kernels), _d(params), _d(out))
    return out


def loss_grad(prob, data, invvar, params, want_grad=True, sgn_override=None, lam=None, W=None, lam_pts=0.0,
              sgn_override_pts=None):
    """Deconvolution loss (Eqs. 10-11, the point-source term when lam_pts != 0) and
    gradient. Returns (loss[3], grad|None)."""
    frame_offsets(prob.n, prob.s, prob.N)
    n, K = _i32(prob.n), _i32(prob.K)
    data, invvar, params = _f64(data), _f64(invvar), _f64(params)
    kernels = _f64(prob.kernels)
    Wv = _f64(prob.W if W is None else W)
    loss = np.zeros(3)
    grad = np.zeros(prob.n_params) if want_grad else None
    so = None
    if sgn_override is not None:
        so = np.ascontiguousarray(sgn_override, dtype=np.int8)
    lib().ora_loss_grad(prob.E, n.ctypes.data_as(_I), K.ctypes.data_as(_I), prob.s, prob.N,
                        prob.M, prob.J, prob.w_stride,
                        ctypes.c_double(prob.lam if lam is None else lam),
                        ctypes.c_double(prob.fwhm), _d(data), _d(invvar), _d(kernels), _d(Wv),
                        _d(params), _d(grad), _d(loss),
                        so.ctypes.data_as(_B) if so is not None else None)
    if lam_pts:
        sp = None if sgn_override_pts is None else np.ascontiguousarray(sgn_override_pts, dtype=np.int8)
        lib().ora_pts_term(prob.E, prob.N, prob.M, prob.J, prob.w_stride, ctypes.c_double(lam_pts),
                           ctypes.c_double(prob.fwhm), _d(Wv), _d(params), _d(grad), _d(loss),
                           sp.ctypes.data_as(_B) if sp is not None else None)
    return loss, grad


def pts_image(prob, params):
    """P = sum_k <a_k> r_k on the N x N grid (Eq. 11, third term), via numpy."""
    N, E, M = prob.N, prob.E, prob.M
    p = _f64(params)
    a = p[N * N + E:N * N + E + E * M].reshape(E, M).mean(axis=0)
    c = p[N * N + E + E * M:].reshape(M, 2)
    sig = sigma_from_fwhm(prob.fwhm)
    Y, X = np.mgrid[0:N, 0:N].astype(np.float64)
    img = np.zeros((N, N))
    for k in range(M):
        img += a[k] * np.exp(-((X - c[k, 0]) ** 2 + (Y - c[k, 1]) ** 2) / (2 * sig * sig)) / (2 * np.pi * sig * sig)
    return img.ravel()


def lambda_pts_estimate(prob, params, lam=None, W=None):
    """App. C estimate of lambda_pts at params."""
    Wv = _f64(prob.W if W is None else W)
    return float(lib().ora_lambda_pts_estimate(prob.E, prob.N, prob.M, prob.J, prob.w_stride,
                                               ctypes.c_double(prob.lam if lam is None else lam),
                                               ctypes.c_double(prob.fwhm), _d(Wv), _d(_f64(params))))


def moffat(N, eta, want_grad=False):
    eta = _f64(eta)
    m = np.zeros(N * N)
    dm = np.zeros(5 * N * N) if want_grad else None
    lib().ora_moffat(N, _d(eta), _d(m), _d(dm))
    return (m, dm) if want_grad else m


def psf_render(N, params):
    params = _f64(params)
    out = np.zeros(N * N)
    lib().ora_psf_render(N, _d(params), _d(out))
    return out


def psf_model(prob, params):
    params = _f64(params)
    out = np.zeros(prob.S * prob.n * prob.n)
    lib().ora_psf_model(prob.S, prob.n, prob.s, prob.N, ctypes.c_double(prob.fwhm), _d(params),
                        _d(out))
    return out


def psf_loss_grad(prob, data, invvar, params, want_grad=True, sgn_override=None, lam=None):
    data, invvar, params = _f64(data), _f64(invvar), _f64(params)
    Wv = _f64(prob.W)
    loss = np.zeros(3)
    grad = np.zeros(prob.n_params) if want_grad else None
    so = None
    if sgn_override is not None:
        so = np.ascontiguousarray(sgn_override, dtype=np.int8)
    lib().ora_psf_loss_grad(prob.S, prob.n, prob.s, prob.N, prob.J, prob.w_stride,
                            ctypes.c_double(prob.lam if lam is None else lam),
                            ctypes.c_double(prob.fwhm), _d(data), _d(invvar), _d(Wv), _d(params),
                            _d(grad), _d(loss), so.ctypes.data_as(_B) if so is not None else None)
    return loss, grad


def noise_variance(n1, K1, s, N, J, kernel1, sigma2_data):
    """Exact per-pixel variance (J x N x N) of Phi^T S_1^T C_up^-1 delta_d (Sec. 2.3)."""
    kernel1, sigma2_data = _f64(kernel1), _f64(sigma2_data)
    out = np.zeros(J * N * N)
    lib().ora_noise_variance(n1, K1, s, N, J, _d(kernel1), _d(sigma2_data), _d(out))
    return out


def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter and a 2-word key (four uint32 words)."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    out = (ctypes.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, out)
    return [int(x) for x in out]


def normal(seed, real, idx):
    """Standard normal draw idx of realization real (Philox4x32-10 + Box-Muller)."""
    return float(lib().ora_normal(ctypes.c_uint64(seed), ctypes.c_uint32(real), ctypes.c_uint32(idx)))


def noise_weights_mc(n1, K1, s, N, J, kernel1, sigma2_data, R, normals=None, seed=0, per_pixel=True):
    """Monte Carlo W (Sec. 2.3): J x N x N (per_pixel) or J values."""
    kernel1, sigma2_data = _f64(kernel1), _f64(sigma2_data)
    out = np.zeros(J * N * N if per_pixel else J)
    nz = None if normals is None else _f64(normals)
    lib().ora_noise_weights_mc(n1, K1, s, N, J, _d(kernel1), _d(sigma2_data), int(R),
                               _d(nz) if nz is not None else None, ctypes.c_uint64(seed),
                               1 if per_pixel else 0, _d(out))
    return out


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays (params, m, v)."""
    assert params.dtype == np.float64 and m.dtype == np.float64 and v.dtype == np.float64
    grad = _f64(grad)
    lr = _f64(np.broadcast_to(lr, params.shape))
    lib().ora_adam_step(ctypes.c_long(params.size), _d(params), _d(grad), _d(m), _d(v), t, _d(lr),
                        ctypes.c_double(beta1), ctypes.c_double(beta2), ctypes.c_double(eps))


def adabelief_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-16, eps_root=1e-16):
    """In-place AdaBelief update of float64 arrays (params, m, v)."""
    assert params.dtype == np.float64 and m.dtype == np.float64 and v.dtype == np.float64
    grad = _f64(grad)
    lr = _f64(np.broadcast_to(lr, params.shape))
    lib().ora_adabelief_step(ctypes.c_long(params.size), _d(params), _d(grad), _d(m), _d(v), t, _d(lr),
                             ctypes.c_double(beta1), ctypes.c_double(beta2), ctypes.c_double(eps),
                             ctypes.c_double(eps_root))


def lbfgs_direction(g, S, Y, count, newest):
    """L-BFGS two-loop recursion: d = -H g from the ring buffers S, Y ([m][n])."""
    g = _f64(g)
    S, Y = _f64(S), _f64(Y)
    m, n = S.shape
    d = np.zeros(n)
    lib().ora_lbfgs_direction(ctypes.c_long(n), _d(g), _d(S), _d(Y), m, count, newest, _d(d))
    return d


def render_scene_xf(n, s, N, M, fwhm, params, xf):
    """Scenes under per-frame transforms xf (E x 3: dx, dy, theta)."""
    n = _i32(n)
    params, xf = _f64(params), _f64(xf)
    out = np.zeros(int(np.sum((s * n.astype(np.int64)) ** 2)))
    lib().ora_render_scene_xf(len(n), n.ctypes.data_as(_I), s, N, M, ctypes.c_double(fwhm), _d(params), _d(xf),
                              _d(out))
    return out


def loss_grad_xf(prob, data, invvar, params, xf, want_grad=True, sgn_override=None, lam=None, W=None):
    """Loss and gradient with per-frame transforms; returns (loss, grad, dL/dxf)."""
    frame_offsets(prob.n, prob.s, prob.N)
    n, K = _i32(prob.n), _i32(prob.K)
    params, xf = _f64(params), _f64(xf)
    Wv = _f64(prob.W if W is None else W)
    loss = np.zeros(3)
    grad = np.zeros(prob.n_params) if want_grad else None
    gxf = np.zeros(3 * prob.E) if want_grad else None
    sp = None if sgn_override is None else np.ascontiguousarray(sgn_override, dtype=np.int8)
    lib().ora_loss_grad_xf(prob.E, n.ctypes.data_as(_I), K.ctypes.data_as(_I), prob.s, prob.N, prob.M, prob.J,
                           prob.w_stride, ctypes.c_double(prob.lam if lam is None else lam),
                           ctypes.c_double(prob.fwhm), _d(_f64(data)), _d(_f64(invvar)), _d(_f64(prob.kernels)),
                           _d(Wv), _d(params), _d(xf), _d(grad), _d(gxf), _d(loss),
                           sp.ctypes.data_as(_B) if sp is not None else None)
    return loss, grad, gxf
