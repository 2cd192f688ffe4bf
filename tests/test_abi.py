"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/starred.h declares, and rejects bad descriptions before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2402_08725_amd import build, starred
    if not os.path.exists(starred.LIB_PATH):
        build.build()
    return starred.lib()


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "starred.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(starred_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = _declared_symbols()
    for required in ["starred_plan_create", "starred_plan_destroy", "starred_set_frames",
                     "starred_render_scene", "starred_convolve_subsample",
                     "starred_convolve_subsample_adj", "starred_starlet_fwd", "starred_starlet_adj",
                     "starred_loss_grad", "starred_step", "starred_last_error", "starred_abi_version"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared_symbols() if not hasattr(L, n)]
    assert not missing, missing
    assert L.starred_abi_version() == 1


def _desc(**kw):
    from paper_2402_08725_amd import starred as st
    sides = np.array(kw.pop("sides", [16, 16]), np.int32)
    ks = np.array(kw.pop("ks", [9, 9]), np.int32)
    d = st.Desc()
    d.mode = kw.pop("mode", 0)
    d.n_frames = kw.pop("n_frames", len(sides))
    d.side_host = sides.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.ksize_host = ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.subsample = kw.pop("s", 2)
    d.grid_side = kw.pop("N", 32)
    d.n_sources = kw.pop("M", 1)
    d.n_scales = kw.pop("J", 3)
    d.w_pixel_stride = kw.pop("w_stride", 0)
    d.conv_algo = kw.pop("conv_algo", 0)
    d.lambda_ = kw.pop("lam", 3.0)
    d.gauss_fwhm = kw.pop("fwhm", 2.0)
    assert not kw
    return d, (sides, ks)


@pytest.mark.parametrize("kw,frag", [
    (dict(n_frames=0), "n_frames"),
    (dict(s=4), "subsample"),
    (dict(J=7), "2^(J-1)"),
    (dict(sides=[20, 16]), "fit the grid"),
    (dict(sides=[16, 16], N=33), "fit the grid"),
    (dict(ks=[0, 9]), "kernel side"),
    (dict(w_stride=2), "w_pixel_stride"),
    (dict(fwhm=0.0), "gauss_fwhm"),
    (dict(lam=-1.0), "lambda"),
    (dict(M=-1), "n_sources"),
    (dict(mode=7), "mode"),
    (dict(conv_algo=9), "conv_algo"),
])
def test_bad_descriptions_are_rejected_before_any_launch(kw, frag):
    L = _lib()
    d, keep = _desc(**kw)
    h = ctypes.c_void_p()
    rc = L.starred_plan_create(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == -1
    assert frag in L.starred_last_error().decode()
    assert not h.value


def test_null_plan_arguments_are_rejected():
    L = _lib()
    assert L.starred_plan_destroy(None) == -1
    assert L.starred_loss_grad(None, None, None, None) == -1
    assert L.starred_time_stage(None, None, 0, 1, None) == -1
    assert L.starred_noise_weights(None, 0, None, 10, 0, None, 1, None) == -1
    assert L.starred_set_lambda_pts(None, ctypes.c_double(1.0)) == -1
    assert L.starred_estimate_lambda_pts(None, None, None) == -1
    assert L.starred_pts_image(None, None, None) == -1
    assert L.starred_lbfgs_create(None, 10, None, None, None) == -1
    assert L.starred_lbfgs_direction(None, None, None, None, 1, 0, 0, None) == -1
    assert L.starred_lbfgs_run(None, None, 1, None, None) == -1
    assert L.starred_lbfgs_destroy(None) == -1
    assert L.starred_set_frames(None, None, None, None, None) == -1
    assert L.starred_steps(None, None, None, None, 1, None, 1, None) == -1


def test_plan_rejects_a_gaussian_wider_than_its_evaluation_box():
    """r is evaluated within +-8 fine pixels of its centre: a FWHM whose mass beyond
    that box is not negligible is refused before anything runs."""
    from paper_2402_08725_amd import starred as st
    L = _lib()
    d, keep = _desc(fwhm=3.5)
    h = ctypes.c_void_p()
    assert L.starred_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == st.EINVAL
    assert b"gauss_fwhm" in L.starred_last_error()
