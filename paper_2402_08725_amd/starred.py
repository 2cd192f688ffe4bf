"""Python binding of libstarred.so (include/starred.h).

Argument marshalling only: every step of the loss and gradient runs in the HIP
kernels of the library. PyTorch supplies device memory (tensors) and streams;
only raw device pointers and the stream handle cross the C ABI.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libstarred.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5
DECONV, PSF = 0, 1
CONV_AUTO, CONV_DIRECT, CONV_FFT = 0, 1, 2

EXPORTED = [
    "starred_plan_create", "starred_plan_destroy", "starred_num_params", "starred_num_data",
    "starred_num_scene", "starred_set_frames", "starred_render_scene",
    "starred_convolve_subsample", "starred_convolve_subsample_adj", "starred_starlet_fwd",
    "starred_starlet_adj", "starred_loss_grad", "starred_step", "starred_steps", "starred_set_graph_mode",
    "starred_conv_algo", "starred_last_error", "starred_abi_version", "starred_set_profiling",
    "starred_profile_read", "starred_psf_model", "starred_loss_grad_plain", "starred_copy_probe",
]
STAGES = ["render", "conv_fwd", "conv_adj", "grad_sums", "starlet", "finalize", "adam", "spectra",
          "graph", "fft_spec", "fft_mcols", "fft_mrows", "fft_rcols", "fft_acols", "fft_arows",
          "fft_fsum", "fft_fused", "direct_fwd", "direct_adj"]


class ClassInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("K", ctypes.c_int32), ("n_frames", ctypes.c_int32),
                ("algo", ctypes.c_int32), ("P", ctypes.c_int32), ("Q", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("pad", ctypes.c_int32), ("tune_ms", ctypes.c_double * 3)]


class Desc(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("n_frames", ctypes.c_int32),
        ("side_host", ctypes.POINTER(ctypes.c_int32)), ("ksize_host", ctypes.POINTER(ctypes.c_int32)),
        ("subsample", ctypes.c_int32), ("grid_side", ctypes.c_int32), ("n_sources", ctypes.c_int32),
        ("n_scales", ctypes.c_int32), ("w_pixel_stride", ctypes.c_int32), ("conv_algo", ctypes.c_int32),
        ("lambda_", ctypes.c_double), ("gauss_fwhm", ctypes.c_double),
    ]


ADAM, ADABELIEF = 0, 1


class AdamHP(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 4), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("rule", ctypes.c_int32), ("eps_root", ctypes.c_float)]


class StarredError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"starred error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libstarred.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.starred_plan_create.argtypes = [ctypes.POINTER(Desc), vp, ctypes.POINTER(vp)]
        L.starred_plan_destroy.argtypes = [vp]
        for f in ["starred_num_params", "starred_num_data", "starred_num_scene"]:
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = i64
        L.starred_set_frames.argtypes = [vp, vp, vp, vp, vp]
        for f in ["starred_render_scene", "starred_convolve_subsample", "starred_convolve_subsample_adj",
                  "starred_starlet_fwd", "starred_starlet_adj"]:
            getattr(L, f).argtypes = [vp, vp, vp]
        L.starred_loss_grad.argtypes = [vp, vp, vp, vp]
        L.starred_step.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(AdamHP), vp]
        L.starred_steps.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(AdamHP), i32, vp]
        L.starred_set_graph_mode.argtypes = [vp, i32]
        L.starred_set_fft_fused.argtypes = [vp, i32]
        L.starred_conv_algo.argtypes = [vp]
        L.starred_num_classes.argtypes = [vp]
        L.starred_get_class_info.argtypes = [vp, i32, ctypes.POINTER(ClassInfo)]
        L.starred_autotune_info.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32),
                                            ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                            ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.starred_set_class_algo.argtypes = [vp, i32, i32, i32]
        L.starred_set_fft_shapes.argtypes = [vp, i32, i32, i32, i32, i32]
        L.starred_set_frame_transforms.argtypes = [vp, vp, vp, i32]
        L.starred_frame_transforms_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
        L.starred_last_error.restype = ctypes.c_char_p
        L.starred_set_profiling.argtypes = [vp, i32]
        L.starred_profile_read.argtypes = [vp, vp, vp]
        L.starred_psf_model.argtypes = [vp, vp, vp]
        L.starred_loss_grad_plain.argtypes = [vp, vp, vp, vp]
        L.starred_copy_probe.argtypes = [vp, vp, vp, ctypes.c_int64]
        L.starred_time_stage.argtypes = [vp, vp, i32, i32, ctypes.POINTER(ctypes.c_double)]
        L.starred_noise_weights.argtypes = [vp, i32, vp, i32, ctypes.c_uint64, vp, i32, vp]
        L.starred_set_lambda_pts.argtypes = [vp, ctypes.c_double]
        L.starred_pts_image.argtypes = [vp, vp, vp]
        L.starred_lbfgs_direction.argtypes = [vp, vp, vp, vp, i32, i32, i32, vp]
        L.starred_lbfgs_create.argtypes = [vp, i32, vp, vp, ctypes.POINTER(vp)]
        L.starred_lbfgs_destroy.argtypes = [vp]
        L.starred_lbfgs_reset.argtypes = [vp]
        L.starred_lbfgs_run.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
        L.starred_estimate_lambda_pts.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.starred_starlet_fwd_noalloc.argtypes = [i32, i32, vp, vp, vp]
        L.starred_lbfgsb_create.argtypes = [ctypes.c_int64, i32, vp, vp, ctypes.c_double, ctypes.c_double, i32,
                                            ctypes.POINTER(vp)]
        L.starred_lbfgsb_destroy.argtypes = [vp]
        L.starred_lbfgsb_iterate.argtypes = [vp, vp, ctypes.c_double, vp, ctypes.POINTER(i32)]
        L.starred_lbfgsb_counts.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise StarredError(rc, lib().starred_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _f32(x, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device=device)


class Plan:
    """A problem plan: frame tables, preprocessed kernels and scratch on one GPU."""

    def __init__(self, mode, sides, ksizes, s, N, M, J, lam, w_stride=0, fwhm=2.0,
                 conv_algo=CONV_AUTO, device="cuda:0"):
        self.device = torch.device(device)
        self.mode = mode
        self.E = len(sides)
        self.s, self.N, self.M, self.J = int(s), int(N), int(M), int(J)
        self._sides = np.ascontiguousarray(sides, dtype=np.int32)
        self._ks = np.ascontiguousarray(ksizes, dtype=np.int32) if ksizes is not None else None
        d = Desc()
        d.mode = mode
        d.n_frames = self.E
        d.side_host = self._sides.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.ksize_host = (self._ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
                        if self._ks is not None else None)
        d.subsample, d.grid_side, d.n_sources, d.n_scales = self.s, self.N, self.M, self.J
        d.w_pixel_stride, d.conv_algo = w_stride, conv_algo
        d.lambda_, d.gauss_fwhm = float(lam), float(fwhm)
        self.stream = torch.cuda.Stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().starred_plan_create(ctypes.byref(d), ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(h)))
        self._h = h
        self.n_params = lib().starred_num_params(h)
        self.n_data = lib().starred_num_data(h)
        self.n_scene = lib().starred_num_scene(h)
        self._bound = ()

    @classmethod
    def for_problem(cls, prob, conv_algo=CONV_AUTO, device="cuda:0", lam=None):
        return cls(DECONV, prob.n, prob.K, prob.s, prob.N, prob.M, prob.J,
                   prob.lam if lam is None else lam, prob.w_stride, prob.fwhm, conv_algo, device)

    @classmethod
    def for_psf(cls, prob, device="cuda:0", lam=None):
        return cls(PSF, [prob.n] * prob.S, None, prob.s, prob.N, 0, prob.J,
                   prob.lam if lam is None else lam, prob.w_stride, prob.fwhm, CONV_AUTO, device)

    def psf_model(self, params):
        """Star models m_k = D(s * a_k r_k) (PSF mode), packed S x n^2."""
        params = _f32(params, self.device)
        out = torch.empty(self.n_data, dtype=torch.float32, device=self.device)
        self._call(lib().starred_psf_model, _ptr(params), _ptr(out))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().starred_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stream ordering with PyTorch's current stream --
    def _call(self, fn, *args):
        # order the plan's stream after the caller's and back; nothing to do when the
        # caller already works on the plan's stream (torch.cuda.stream(plan.stream))
        cur = torch.cuda.current_stream(self.device)
        same = cur.cuda_stream == self.stream.cuda_stream
        if not same:
            self.stream.wait_stream(cur)
        with torch.cuda.device(self.device):
            rc = fn(self._h, *args)
        if not same:
            cur.wait_stream(self.stream)
        _check(rc)

    @property
    def conv_algo(self):
        return lib().starred_conv_algo(self._h)

    def classes(self):
        """Shape classes: dicts of n, K, n_frames, algo, P, Q, fused."""
        nc = lib().starred_num_classes(self._h)
        _check(min(nc, 0))
        out = []
        for c in range(nc):
            ci = ClassInfo()
            _check(lib().starred_get_class_info(self._h, c, ctypes.byref(ci)))
            d = {k: getattr(ci, k) for k, _ in ClassInfo._fields_ if k not in ("pad", "tune_ms")}
            d["tune_ms"] = [float(v) for v in ci.tune_ms]
            out.append(d)
        return out

    def autotune_info(self):
        """Host ms of the last autotuning, whether it came from the cache, launch shapes."""
        ms, cached = ctypes.c_double(0.0), ctypes.c_int32(0)
        ab, lg, af, sf, pl = (ctypes.c_int32(0) for _ in range(5))
        _check(lib().starred_autotune_info(self._h, ctypes.byref(ms), ctypes.byref(cached), ctypes.byref(ab),
                                           ctypes.byref(lg), ctypes.byref(af), ctypes.byref(sf), ctypes.byref(pl)))
        return {"wall_ms": ms.value, "cached": bool(cached.value), "adj_blocks": ab.value,
                "line_groups": lg.value, "adj_frames": af.value, "split_forward": sf.value,
                "prior_late": pl.value}

    def set_frame_transforms(self, xf, grad_out=None, algo=CONV_AUTO):
        """Per-frame (dx, dy, theta) transforms (E x 3), or None to clear them; grad_out
        (float32 device tensor of E x 3) receives dL/d(dx, dy, theta) in loss_grad; algo:
        how the transformed frames are convolved (CONV_AUTO, CONV_DIRECT or CONV_FFT)."""
        if xf is None:
            self._xf = None
            self._call(lib().starred_set_frame_transforms, None, None, ctypes.c_int32(CONV_AUTO))
            return None
        t = _f32(xf, self.device)
        g = grad_out if grad_out is not None else torch.zeros(3 * self.E, dtype=torch.float32, device=self.device)
        self._call(lib().starred_set_frame_transforms, _ptr(t), _ptr(g), ctypes.c_int32(int(algo)))
        self._xf = (t, g)  # referenced by the plan
        return g

    def frame_transforms_info(self):
        """(algo, {"direct": ms, "fft": ms}) of the transformed frames' convolution."""
        a = ctypes.c_int32(0)
        ms = (ctypes.c_double * 2)()
        _check(lib().starred_frame_transforms_info(self._h, ctypes.byref(a), ms))
        return a.value, {"direct": ms[0], "fft": ms[1]}

    def set_class_algo(self, c, algo, fused=True):
        """Force shape class c onto CONV_DIRECT or CONV_FFT (one-launch forward if fused)."""
        _check(lib().starred_set_class_algo(self._h, int(c), int(algo), 1 if fused else 0))

    def set_fft_shapes(self, adj_frames=0, adj_blocks=0, line_groups=0, split_forward=-1, prior_late=-1):
        """Launch shapes of the FFT path (0, or -1 for the two switches, keeps the current value)."""
        _check(lib().starred_set_fft_shapes(self._h, int(adj_frames), int(adj_blocks), int(line_groups),
                                            int(split_forward), int(prior_late)))

    def fused_classes(self):
        """(n, K) of the classes whose forward is the one-launch form."""
        return {(c["n"], c["K"]) for c in self.classes() if c["algo"] == CONV_FFT and c["fused"]}

    def set_frames(self, data, invvar, psf, W):
        t = [_f32(x, self.device) if x is not None else None for x in (data, invvar, psf, W)]
        self._call(lib().starred_set_frames, *[_ptr(x) for x in t])
        # keep the memory alive while the plan references it (the old arrays stay bound
        # when the call fails)
        self._bound = tuple(t)

    def render_scene(self, params):
        params = _f32(params, self.device)
        out = torch.empty(self.n_scene if self.mode == DECONV else self.N * self.N,
                          dtype=torch.float32, device=self.device)
        self._call(lib().starred_render_scene, _ptr(params), _ptr(out))
        return out

    def convolve_subsample(self, scene):
        scene = _f32(scene, self.device)
        out = torch.empty(self.n_data, dtype=torch.float32, device=self.device)
        self._call(lib().starred_convolve_subsample, _ptr(scene), _ptr(out))
        return out

    def convolve_subsample_adj(self, resid):
        resid = _f32(resid, self.device)
        out = torch.empty(self.n_scene, dtype=torch.float32, device=self.device)
        self._call(lib().starred_convolve_subsample_adj, _ptr(resid), _ptr(out))
        return out

    def starlet_fwd(self, img):
        img = _f32(img, self.device)
        out = torch.empty(self.J * self.N * self.N, dtype=torch.float32, device=self.device)
        self._call(lib().starred_starlet_fwd, _ptr(img), _ptr(out))
        return out

    def starlet_adj(self, coeffs):
        coeffs = _f32(coeffs, self.device)
        out = torch.empty(self.N * self.N, dtype=torch.float32, device=self.device)
        self._call(lib().starred_starlet_adj, _ptr(coeffs), _ptr(out))
        return out

    def loss_grad(self, params, want_grad=True, grad_out=None, loss_out=None):
        """Returns (loss double[3] tensor, grad float32 tensor or None)."""
        params = _f32(params, self.device)
        loss = loss_out if loss_out is not None else torch.empty(3, dtype=torch.float64, device=self.device)
        grad = None
        if want_grad:
            grad = grad_out if grad_out is not None else torch.empty(self.n_params, dtype=torch.float32,
                                                                      device=self.device)
        self._call(lib().starred_loss_grad, _ptr(params), _ptr(grad), _ptr(loss))
        return loss, grad

    def loss_grad_plain(self, params, want_grad=True, grad_out=None, loss_out=None):
        """The unfused per-epoch baseline (same results, one launch per operator per frame)."""
        params = _f32(params, self.device)
        loss = loss_out if loss_out is not None else torch.empty(3, dtype=torch.float64, device=self.device)
        grad = None
        if want_grad:
            grad = grad_out if grad_out is not None else torch.empty(self.n_params, dtype=torch.float32,
                                                                      device=self.device)
        self._call(lib().starred_loss_grad_plain, _ptr(params), _ptr(grad), _ptr(loss))
        return loss, grad

    def step(self, params, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, loss_out=None, rule=ADAM,
             eps_root=0.0):
        """One optimiser step (Adam or AdaBelief) in place on (params, m, v); returns the
        loss at the old params."""
        hp = AdamHP()
        for i in range(4):
            hp.lr[i] = float(lr[i])
        hp.beta1, hp.beta2, hp.eps = beta1, beta2, eps
        hp.rule, hp.eps_root = int(rule), float(eps_root)
        loss = loss_out if loss_out is not None else torch.empty(3, dtype=torch.float64, device=self.device)
        self._call(lib().starred_step, _ptr(params), _ptr(m), _ptr(v), int(t), ctypes.byref(hp), _ptr(loss))
        return loss

    def steps(self, params, m, v, t, lr, n, beta1=0.9, beta2=0.999, eps=1e-8, loss_out=None, rule=ADAM,
              eps_root=0.0):
        """n consecutive optimiser steps t .. t+n-1 (several per graph launch in graph mode);
        returns the last step's loss."""
        hp = AdamHP()
        for i in range(4):
            hp.lr[i] = float(lr[i])
        hp.beta1, hp.beta2, hp.eps = beta1, beta2, eps
        hp.rule, hp.eps_root = int(rule), float(eps_root)
        loss = loss_out if loss_out is not None else torch.empty(3, dtype=torch.float64, device=self.device)
        self._call(lib().starred_steps, _ptr(params), _ptr(m), _ptr(v), int(t), ctypes.byref(hp), int(n),
                   _ptr(loss))
        return loss

    def set_profiling(self, enable: bool):
        _check(lib().starred_set_profiling(self._h, int(bool(enable))))

    def profile_read(self):
        """Per-stage summed milliseconds and launch counts since the last read."""
        ms = np.zeros(len(STAGES), np.float64)
        cnt = np.zeros(len(STAGES), np.int64)
        _check(lib().starred_profile_read(self._h, ctypes.c_void_p(ms.ctypes.data),
                                          ctypes.c_void_p(cnt.ctypes.data)))
        return {name: {"ms": float(ms[i]), "count": int(cnt[i])} for i, name in enumerate(STAGES)}

    def noise_weights(self, sigma2_data, n_real, seed=0, normals=None, per_pixel=True, frame=0):
        """W by Monte Carlo noise propagation (Sec. 2.3): J x N x N (per_pixel) or J values."""
        sig = _f32(sigma2_data, self.device)
        nz = _f32(normals, self.device) if normals is not None else None
        out = torch.empty(self.J * self.N * self.N if per_pixel else self.J, dtype=torch.float32,
                          device=self.device)
        self._call(lib().starred_noise_weights, ctypes.c_int32(frame), _ptr(sig), ctypes.c_int32(int(n_real)),
                   ctypes.c_uint64(int(seed)), _ptr(nz), ctypes.c_int32(1 if per_pixel else 0), _ptr(out))
        return out

    def time_stage(self, params, stage: str, reps: int = 50) -> float:
        """Average device milliseconds of one stage's launches run back to back."""
        params = _f32(params, self.device)
        ms = ctypes.c_double(0.0)
        self._call(lib().starred_time_stage, _ptr(params), ctypes.c_int32(STAGES.index(stage)),
                   ctypes.c_int32(int(reps)), ctypes.byref(ms))
        return ms.value

    def copy_probe(self, src, dst):
        """Plain device copy (memory-counter calibration)."""
        self._call(lib().starred_copy_probe, _ptr(src), _ptr(dst), int(src.numel()))

    def set_lambda_pts(self, lambda_pts: float):
        """Weight of the point-source prior (Eq. 11, third term); 0 leaves it out."""
        _check(lib().starred_set_lambda_pts(self._h, ctypes.c_double(float(lambda_pts))))

    def pts_image(self, params):
        """P = sum_k <a_k> r_k on the N x N grid (Eq. 11, third term)."""
        params = _f32(params, self.device)
        out = torch.empty(self.N * self.N, dtype=torch.float32, device=self.device)
        self._call(lib().starred_pts_image, _ptr(params), _ptr(out))
        return out

    def estimate_lambda_pts(self, params) -> float:
        """App. C estimate of lambda_pts at params."""
        params = _f32(params, self.device)
        out = ctypes.c_double(0.0)
        self._call(lib().starred_estimate_lambda_pts, _ptr(params), ctypes.byref(out))
        return out.value

    def lbfgs_direction(self, grad, S, Y, count, newest):
        """d = -H grad by the two-loop recursion over the ring buffers S, Y ([m][n])."""
        g = _f32(grad, self.device)
        S, Y = _f32(S, self.device), _f32(Y, self.device)
        d = torch.empty_like(g)
        self._call(lib().starred_lbfgs_direction, _ptr(g), _ptr(S), _ptr(Y), int(S.shape[0]), int(count),
                   int(newest), _ptr(d))
        return d

    def lbfgs(self, m=10, lo=None, hi=None):
        """An L-BFGS state on this plan's loss (optional box bounds)."""
        return LBFGS(self, m, lo, hi)

    def set_fft_fused(self, enable: bool):
        """FFT path: one-launch forward for frames whose spectra fit in LDS (default on)."""
        _check(lib().starred_set_fft_fused(self._h, 1 if enable else 0))

    def set_graph_mode(self, enable: bool):
        _check(lib().starred_set_graph_mode(self._h, int(bool(enable))))


def starlet_fwd_noalloc(N, J, img, out):
    """Phi^T of img (N x N, float32 device tensor) into out (J N^2), without a plan and
    without allocating device memory (the library's fixed working array)."""
    stream = torch.cuda.current_stream(img.device)
    with torch.cuda.device(img.device):
        _check(lib().starred_starlet_fwd_noalloc(int(N), int(J), _ptr(img), _ptr(out),
                                                 ctypes.c_void_p(stream.cuda_stream)))
    return out


LBFGSB_FG, LBFGSB_NEW_X, LBFGSB_CONVERGED, LBFGSB_ABNORMAL = 1, 2, 3, 4


class LBFGSB:
    """The library's L-BFGS-B iteration on the host (reverse communication): any
    function of float64 vectors can drive it."""

    def __init__(self, n, m=10, lo=None, hi=None, factr=1e7, pgtol=1e-5, maxls=20):
        self.n = int(n)
        self._lo = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64)
        self._hi = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().starred_lbfgsb_create(self.n, int(m), _np_ptr(self._lo), _np_ptr(self._hi), float(factr),
                                           float(pgtol), int(maxls), ctypes.byref(h)))
        self._h = h

    def minimize(self, fun, x0, max_iter, callback=None):
        """fun(x) -> (f, g). Returns (x, f, task, iterations, evaluations); callback(x)
        after every iteration."""
        x = np.ascontiguousarray(x0, dtype=np.float64).copy()
        task = ctypes.c_int32(0)
        _check(lib().starred_lbfgsb_iterate(self._h, _np_ptr(x), 0.0, None, ctypes.byref(task)))
        f, g = 0.0, np.zeros(self.n)
        it = 0
        while it < max_iter:
            if task.value == LBFGSB_FG:
                f, g = fun(x)
                g = np.ascontiguousarray(g, dtype=np.float64)
            _check(lib().starred_lbfgsb_iterate(self._h, _np_ptr(x), float(f), _np_ptr(g), ctypes.byref(task)))
            if task.value == LBFGSB_NEW_X:
                it += 1
                if callback:
                    callback(x.copy())
            elif task.value in (LBFGSB_CONVERGED, LBFGSB_ABNORMAL):
                if task.value == LBFGSB_CONVERGED and callback:
                    callback(x.copy())
                break
        ni, ne = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().starred_lbfgsb_counts(self._h, ctypes.byref(ni), ctypes.byref(ne)))
        return x, f, task.value, ni.value, ne.value

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().starred_lbfgsb_destroy(self._h)
                self._h = None
        except Exception:
            pass


def _np_ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class StarredLoss(torch.autograd.Function):
    """Loss of Eq. (11) (or Eq. (7)) as an autograd function whose backward is
    the library's hand-written adjoint: forward calls loss_grad and keeps the
    gradient, backward scales it by the incoming gradient."""

    @staticmethod
    def forward(ctx, params, plan):
        loss, grad = plan.loss_grad(params.detach())
        ctx.save_for_backward(grad)
        return loss[2].clone()

    @staticmethod
    def backward(ctx, grad_output):
        (grad,) = ctx.saved_tensors
        return (grad_output.to(grad.dtype) * grad), None


def starred_loss(params, plan):
    return StarredLoss.apply(params, plan)


class LBFGS:
    """L-BFGS iterations on a plan's loss (state and history on the device)."""

    def __init__(self, plan, m=10, lo=None, hi=None):
        self.plan = plan
        self._lo = _f32(lo, plan.device) if lo is not None else None
        self._hi = _f32(hi, plan.device) if hi is not None else None
        h = ctypes.c_void_p()
        _check(lib().starred_lbfgs_create(plan._h, int(m), _ptr(self._lo), _ptr(self._hi), ctypes.byref(h)))
        self._h = h

    def run(self, x, n_iter):
        """n_iter iterations in place on x (float32 device tensor); returns (loss, evaluations)."""
        loss = ctypes.c_double(0.0)
        ev = ctypes.c_int32(0)
        self.plan._call(lambda _, *a: lib().starred_lbfgs_run(self._h, *a), _ptr(x), int(n_iter),
                        ctypes.byref(loss), ctypes.byref(ev))
        return loss.value, ev.value

    def reset(self):
        _check(lib().starred_lbfgs_reset(self._h))

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().starred_lbfgs_destroy(self._h)
                self._h = None
        except Exception:
            pass
