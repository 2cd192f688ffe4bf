"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: loss relative error <= 1e-6; gradient relative error (L2, per parameter
block and overall) <= 1e-4, after substituting the device's own sign for starlet
coefficients that are zero up to rounding (oracle/parity.py). Operators alone
are compared element by element against the oracle relative to the largest
value of each frame.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as ora
from oracle import parity
from paper_2402_08725_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _st():
    from paper_2402_08725_amd import starred as st
    return st


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _data(prob, seed=0):
    rng = np.random.default_rng(seed)
    m = ora.forward_model(prob, prob.params_true)
    d, w = synth.add_noise(m, rng)
    return d, w, rng


def _plan(prob, d, w, algo=0):
    st = _st()
    plan = st.Plan.for_problem(prob, conv_algo=algo)
    plan.set_frames(d, w, prob.kernels, prob.W)
    return plan


def _frames(arr, sizes):
    off = 0
    for n in sizes:
        yield arr[off:off + n * n]
        off += n * n


def _check_frames(got, ref, sizes, tol):
    for i, (g, r) in enumerate(zip(_frames(got, sizes), _frames(ref, sizes))):
        scale = max(np.abs(r).max(), 1e-30)
        err = np.abs(g - r).max() / scale
        assert err <= tol, (i, err)


SMALL = [
    # seed, E, sides, K, s, N, M, J
    (101, 3, [16, 24, 8], [15, 16, 5], 2, 48, 2, 4),
    (102, 4, [12, 20, 36, 8], [9, 32, 20, 3], 1, 36, 1, 3),
    (103, 3, [8, 12, 16], [13, 24, 6], 3, 48, 3, 4),
    (104, 2, [40, 33], [64, 31], 2, 80, 2, 5),
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: f"seed{c[0]}")
def test_render_scene(case):
    seed, E, sides, K, s, N, M, J = case
    prob = synth.make_small_deconv(seed, E, sides, K, s, N, M, J)
    d, w, rng = _data(prob)
    plan = _plan(prob, d, w)
    p = synth.eval_point(prob, "near", rng)
    _say(f"render {seed}")
    got = plan.render_scene(p).cpu().numpy()
    ref = ora.render_scene(prob.n, s, N, M, prob.fwhm, p)
    _check_frames(got, ref, [s * n for n in sides], 2e-6)


ALGOS = [1, 2]  # direct, FFT
ALGO_ID = {1: "direct", 2: "fft"}


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
@pytest.mark.parametrize("case", SMALL, ids=lambda c: f"seed{c[0]}")
def test_convolve_subsample_and_adjoint(case, algo):
    seed, E, sides, K, s, N, M, J = case
    prob = synth.make_small_deconv(seed, E, sides, K, s, N, M, J)
    d, w, rng = _data(prob)
    plan = _plan(prob, d, w, algo)
    assert plan.conv_algo == algo
    scene = synth.f32(rng.standard_normal(prob.fine_size) * 100)
    _say(f"conv {seed} {ALGO_ID[algo]}")
    got = plan.convolve_subsample(scene).cpu().numpy()
    ref = ora.conv_sub(prob.n, prob.K, s, prob.kernels, scene)
    _check_frames(got, ref, sides, 1e-5)
    resid = synth.f32(rng.standard_normal(prob.data_size))
    gota = plan.convolve_subsample_adj(resid).cpu().numpy()
    refa = ora.conv_sub_adj(prob.n, prob.K, s, prob.kernels, resid)
    _check_frames(gota, refa, [s * n for n in sides], 1e-5)
    # FP32 dot-product identity of the device operators
    lhs = np.dot(got.astype(np.float64), resid)
    rhs = np.dot(scene, gota.astype(np.float64))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(got) * np.linalg.norm(resid)


# (128, 7) reaches level 6, whose composite taps are read from the padded table rather
# than compiled in; (256, 8), (300, 5) and (300, 7) run the cascade (eight scales, and grids
# above 256, are beyond the composite filters); in (256, 8) and (300, 7) the holes of the
# top levels exceed the 16-pixel tiles, so those levels stage only the taps' lines (with
# ragged tiles and mirror images at both edges in (300, 7))
@pytest.mark.parametrize("N,J", [(48, 4), (64, 3), (128, 6), (33, 5), (128, 7), (256, 8), (300, 5), (300, 7)])
def test_starlet_forward_and_adjoint(N, J):
    prob = synth.make_small_deconv(7, 1, [N], [5], 1, N, 1, J)
    d, w, rng = _data(prob)
    plan = _plan(prob, d, w)
    img = synth.f32(rng.standard_normal(N * N) * 10)
    _say(f"starlet {N} {J}")
    got = plan.starlet_fwd(img).cpu().numpy().reshape(J, -1)
    ref = ora.starlet_fwd(N, J, img).reshape(J, -1)
    for j in range(J):
        assert np.abs(got[j] - ref[j]).max() <= 2e-6 * np.abs(ref).max(), j
    z = synth.f32(rng.standard_normal(J * N * N))
    gota = plan.starlet_adj(z).cpu().numpy()
    refa = ora.starlet_adj(N, J, z)
    assert np.abs(gota - refa).max() <= 2e-6 * np.abs(refa).max()


def _compare_loss_grad(prob, d, w, p, plan, label, loss_tol=1e-6, grad_tol=1e-4):
    loss, grad = plan.loss_grad(p)
    loss = loss.cpu().numpy()
    grad = grad.cpu().numpy().astype(np.float64)
    NN = prob.N * prob.N
    alpha_dev = plan.starlet_fwd(p[:NN]).cpu().numpy()
    so, nsub = parity.tie_override(prob.N, prob.J, p[:NN], alpha_dev)
    lo, go = ora.loss_grad(prob, d, w, p, sgn_override=so)
    rl = abs(loss[2] - lo[2]) / abs(lo[2])
    blocks = {k: parity.rel_err(parity.deconv_blocks(prob, grad)[k], v)
              for k, v in parity.deconv_blocks(prob, go).items() if np.linalg.norm(v) > 0}
    rg = parity.rel_err(grad, go)
    _say(f"{label}: loss rel {rl:.2e} (chi {abs(loss[0]-lo[0])/max(abs(lo[0]),1e-300):.2e}, "
         f"l1 {abs(loss[1]-lo[1])/max(abs(lo[1]),1e-300):.2e}); grad rel {rg:.2e} {blocks}; ties {nsub}")
    assert rl <= loss_tol
    assert rg <= grad_tol
    for k, v in blocks.items():
        assert v <= grad_tol, (k, v)
    return loss, grad


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_stage_timing_leaves_results_unchanged(algo):
    """Timing a stage alone re-runs its launches on the plan's buffers; the next
    evaluation must still give bit-identical results, and stages of the other
    algorithm are refused."""
    st = _st()
    prob = synth.make_deconv(2, E=6)
    d, w, rng = _data(prob, seed=5)
    plan = _plan(prob, d, w, algo=algo)
    p = torch.as_tensor(synth.eval_point(prob, "near", rng), dtype=torch.float32, device="cuda")
    l0, g0 = plan.loss_grad(p)
    own = (["spectra", "fft_fused", "fft_spec", "fft_mcols", "fft_mrows", "fft_rcols", "fft_acols",
            "fft_fsum", "fft_arows", "starlet"] if algo == 2 else ["render", "conv_fwd", "conv_adj", "grad_sums", "starlet"])
    for stage in own:
        ms = plan.time_stage(p, stage, reps=3)
        _say(f"{ALGO_ID[algo]} {stage}: {ms * 1e3:.1f} us")
        assert 0.0 <= ms < 1e3
    other = "conv_fwd" if algo == 2 else "fft_acols"
    with pytest.raises(st.StarredError):
        plan.time_stage(p, other, reps=1)
    with pytest.raises(st.StarredError):
        plan.time_stage(p, "adam", reps=1)
    l1, g1 = plan.loss_grad(p)
    assert torch.equal(l0, l1) and torch.equal(g0, g1)


LG_CASES = [
    ("cfg1", lambda: synth.make_deconv(1)),
    ("cfg2_E6", lambda: synth.make_deconv(2, E=6)),
    ("cfg4_mini", lambda: synth.make_deconv(4, E=12, sizes=[16, 24, 32, 48], N=96)),
    ("small_s3", lambda: synth.make_small_deconv(103, 3, [8, 12, 16], [13, 24, 6], 3, 48, 3, 4)),
    ("small_s1_wmap", lambda: synth.make_small_deconv(105, 3, [20, 12, 32], [9, 16, 21], 1, 32, 2, 4,
                                                      w_stride=1)),
]


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
@pytest.mark.parametrize("name,make", LG_CASES, ids=[c[0] for c in LG_CASES])
@pytest.mark.parametrize("point", ["init", "near"])
def test_loss_grad_parity(name, make, point, algo):
    prob = make()
    d, w, rng = _data(prob, seed=sum(map(ord, name)))
    plan = _plan(prob, d, w, algo)
    p = synth.eval_point(prob, point, rng)
    _compare_loss_grad(prob, d, w, p, plan, f"{name}/{point}/{ALGO_ID[algo]}")


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_loss_grad_parity_seven_scales(algo):
    """Seven starlet scales on a 128 grid: the prior's level-6 filters come from the
    padded tap table (levels 1-5 are compiled in); one shape class covering the whole
    grid, so on the FFT path the prior's passes ride in the evaluation's own launches
    (with the gradient too)."""
    prob = synth.make_small_deconv(211, 3, [64, 64, 64], [31, 31, 31], 2, 128, 2, 7)
    d, w, rng = _data(prob, seed=211)
    plan = _plan(prob, d, w, algo)
    assert len(plan.classes()) == 1
    p = synth.eval_point(prob, "near", rng)
    _compare_loss_grad(prob, d, w, p, plan, f"J7/{ALGO_ID[algo]}")


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_widest_accepted_gaussian(algo):
    """r_k at the widest FWHM a plan accepts (3 fine px: the +-8 px box the kernels
    evaluate it in holds 6.3 sigma): the render and the loss and gradient against the
    oracle's untruncated Gaussian, s = 3 with three sources."""
    prob = synth.make_small_deconv(103, 3, [8, 12, 16], [13, 24, 6], 3, 48, 3, 4)
    prob.fwhm = 3.0
    d, w, rng = _data(prob, seed=303)
    plan = _plan(prob, d, w, algo)
    p = synth.eval_point(prob, "near", rng)
    got = plan.render_scene(p).cpu().numpy()
    ref = ora.render_scene(prob.n, prob.s, prob.N, prob.M, prob.fwhm, p)
    _check_frames(got, ref, [prob.s * n for n in prob.n], 2e-6)
    _compare_loss_grad(prob, d, w, p, plan, f"fwhm3/{ALGO_ID[algo]}")


@pytest.mark.parametrize("s", [1, 2, 3])
def test_many_sources_fft(s):
    """More than sixteen point sources (the spectral product's source-major form) at
    s = 1, 2 and 3, five ragged frames (a frame group of four and one of one), FFT path,
    against the oracle."""
    N = {1: 40, 2: 64, 3: 72}[s]
    prob = synth.make_small_deconv(340 + s, 5, [N // s - 8, N // s], [11, 16], s, N, 17, 4)
    d, w, rng = _data(prob, seed=341 + s)
    plan = _plan(prob, d, w, 2)
    p = synth.eval_point(prob, "near", rng)
    _compare_loss_grad(prob, d, w, p, plan, f"M17/s{s}/fft")


@pytest.mark.parametrize("E", [1, 3, 5])
def test_loss_grad_parity_few_epochs_fft(E):
    """The frequency-domain adjoint with fewer frame chunks than the chunk sums' runs per
    bin (1 or 2 chunks), and a last chunk holding a single frame (odd E)."""
    prob = synth.make_deconv(2, E=E)
    d, w, rng = _data(prob, seed=40 + E)
    plan = _plan(prob, d, w, 2)
    p = synth.eval_point(prob, "near", rng)
    _compare_loss_grad(prob, d, w, p, plan, f"cfg2_E{E}/fft")


@pytest.mark.parametrize("name,make", [LG_CASES[1], LG_CASES[2], LG_CASES[3]], ids=["cfg2_E6", "cfg4_mini",
                                                                                   "small_s3"])
def test_fft_line_passes_without_the_fused_forward(name, make):
    """The FFT forward through the batched line passes (the path of frames too large
    for the one-launch forward) on shapes that would otherwise take the one-launch
    kernel: both must match the oracle."""
    prob = make()
    d, w, rng = _data(prob, seed=13)
    plan = _plan(prob, d, w, algo=2)
    p = synth.eval_point(prob, "near", rng)
    _, g_fused = _compare_loss_grad(prob, d, w, p, plan, f"{name}/fused")
    plan.set_fft_fused(False)
    _, g_lines = _compare_loss_grad(prob, d, w, p, plan, f"{name}/line passes")
    plan.set_fft_fused(True)
    assert parity.rel_err(g_fused, g_lines) <= 1e-4


def test_loss_grad_cfg2_full_size_both_algorithms_and_autotune():
    prob = synth.make_deconv(2)
    _say("cfg2 full: oracle data")
    d, w, rng = _data(prob, seed=2)
    p = synth.eval_point(prob, "near", rng)
    NN = prob.N * prob.N
    so, _ = parity.tie_override(prob.N, prob.J, p[:NN], _plan(prob, d, w, 1).starlet_fwd(p[:NN]).cpu().numpy())
    lo, go = ora.loss_grad(prob, d, w, p, sgn_override=so)
    for algo in (1, 2, 0):
        plan = _plan(prob, d, w, algo)
        loss, grad = plan.loss_grad(p)
        loss = loss.cpu().numpy()
        grad = grad.cpu().numpy().astype(np.float64)
        rl = abs(loss[2] - lo[2]) / abs(lo[2])
        blocks = {k: parity.rel_err(parity.deconv_blocks(prob, grad)[k], v)
                  for k, v in parity.deconv_blocks(prob, go).items()}
        _say(f"cfg2 full algo {algo} -> {plan.conv_algo}: loss rel {rl:.2e} grad {blocks}")
        assert rl <= 1e-6
        for k, v in blocks.items():
            assert v <= 1e-4, (algo, k, v)


def test_forward_only_matches_and_is_deterministic():
    prob = synth.make_deconv(2, E=5)
    d, w, rng = _data(prob, seed=3)
    plan = _plan(prob, d, w)
    p = synth.eval_point(prob, "near", rng)
    l1, g1 = plan.loss_grad(p)
    l2, g2 = plan.loss_grad(p)
    l3, _ = plan.loss_grad(p, want_grad=False)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    assert torch.equal(l1, l3)


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_autograd_function_and_directional_differences(algo):
    st = _st()
    prob = synth.make_deconv(1)
    d, w, rng = _data(prob, seed=4)
    plan = st.Plan.for_problem(prob, lam=0.0, conv_algo=algo)
    plan.set_frames(d, w, prob.kernels, prob.W)
    p0 = synth.eval_point(prob, "near", rng)
    x = torch.tensor(p0, dtype=torch.float32, device="cuda", requires_grad=True)
    L = st.starred_loss(x, plan)
    (2.5 * L).backward()
    _, g = plan.loss_grad(p0)
    assert torch.allclose(x.grad, 2.5 * g)
    # chi^2 is exactly quadratic in (h, Gamma, a): central differences are exact
    NN, E, M = prob.N ** 2, prob.E, prob.M
    # (h, Gamma, a): large steps, the differences being exact, so that the FP32
    # rounding of the two loss values stays small against their difference
    for block, sl, eps in [("h", slice(0, NN), 10.0), ("Gamma", slice(NN, NN + E), 10.0),
                           ("a", slice(NN + E, NN + E + E * M), 100.0),
                           ("c", slice(NN + E + E * M, None), 1e-2)]:
        delta = np.zeros(prob.n_params)
        delta[sl] = rng.standard_normal(delta[sl].shape)
        lp = plan.loss_grad(synth.f32(p0 + eps * delta), want_grad=False)[0][2].item()
        lm = plan.loss_grad(synth.f32(p0 - eps * delta), want_grad=False)[0][2].item()
        # the perturbed points are rounded to FP32: use the exact steps taken
        dp = synth.f32(p0 + eps * delta) - synth.f32(p0 - eps * delta)
        fd = (lp - lm)
        an = float(np.dot(g.cpu().numpy().astype(np.float64), dp))
        # the loss values differ in their FP32 model rounding (more steps through the
        # transforms on the FFT path), which the difference of two losses exposes
        tol = 1e-3 if block == "c" else (1e-4 if algo == 1 else 3e-4)
        _say(f"fd {block}: fd {fd:.6e} analytic {an:.6e}")
        assert abs(fd - an) <= tol * abs(an) + 1e-9, block


ADAM200_LOSS_BAR = 1e-3


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_adam_200_steps_against_oracle(algo):
    """Direct path: separate update launch; FFT path: update fused into the final
    reduction launch, step counter advanced by the first launch."""
    st = _st()
    prob = synth.make_deconv(1)
    d, w, rng = _data(prob, seed=5)
    p0 = synth.eval_point(prob, "init", rng)
    lrv = prob.lr_vector()
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    plan = _plan(prob, d, w, algo=algo)
    x = torch.tensor(p0, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(x)
    v = torch.zeros_like(x)
    po = p0.copy()
    mo = np.zeros_like(po)
    vo = np.zeros_like(po)
    steps = 200
    NN = prob.N ** 2
    nties = 0
    for t in range(1, steps + 1):
        plan.step(x, m, v, t, lr4)
        # the oracle's subgradient takes the device's sign on coefficients that are
        # zero up to rounding (several subgradients are correct there, and Adam's
        # normalised step would turn an arbitrary choice into a full-lr step)
        so, nsub = parity.tie_override(prob.N, prob.J, po[:NN], plan.starlet_fwd(po[:NN]).cpu().numpy())
        nties += nsub
        _, go = ora.loss_grad(prob, d, w, po, sgn_override=so)
        ora.adam_step(po, go, mo, vo, t, lrv)
    lg = plan.loss_grad(x)[0].cpu().numpy()
    lo, _ = ora.loss_grad(prob, d, w, po, want_grad=False)
    xf = x.cpu().numpy().astype(np.float64)
    cdev = xf[-2 * prob.M:]
    cora = po[-2 * prob.M:]
    _say(f"adam200: loss dev {lg[2]:.6e} oracle {lo[2]:.6e} rel {abs(lg[2] - lo[2]) / abs(lo[2]):.2e}; "
         f"c dev {cdev} oracle {cora}; tied coefficients over the run {nties}")
    # The bar on the final loss is ADAM200_LOSS_BAR: the oracle's own 200-step final
    # loss moves by up to 2.4e-4 when its gradients carry relative perturbations of
    # 1e-6 (the FP32 path's gradient error), because the l1 subgradient turns a
    # coefficient's zero crossing a step earlier or later into a different path
    # (tests/test_tolerances.py pins that spread on the CPU).
    assert abs(lg[2] - lo[2]) / abs(lo[2]) <= ADAM200_LOSS_BAR
    assert np.abs(cdev - cora).max() <= 0.01


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_steps_equal_repeated_single_steps(algo, graph):
    """starred_steps(n) runs the same launches as n calls of starred_step (several
    steps per graph launch in graph mode, then single-step graphs for the rest):
    bitwise the same parameters, moments and last loss, also across the boundary
    between two calls (the device step counter carries on)."""
    prob = synth.make_deconv(2, E=6)
    d, w, rng = _data(prob, seed=21)
    p0 = synth.eval_point(prob, "init", rng)
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    runs = []
    for many in (False, True):
        plan = _plan(prob, d, w, algo=algo)
        plan.set_graph_mode(graph)
        x = torch.tensor(p0, dtype=torch.float32, device="cuda")
        m = torch.zeros_like(x)
        v = torch.zeros_like(x)
        loss = torch.empty(3, dtype=torch.float64, device="cuda")
        if many:
            plan.steps(x, m, v, 1, lr4, 11, loss_out=loss)   # one 8-step graph and 3 single steps
            plan.steps(x, m, v, 12, lr4, 9, loss_out=loss)
        else:
            for t in range(1, 21):
                plan.step(x, m, v, t, lr4, loss_out=loss)
        torch.cuda.synchronize()
        runs.append((x.clone(), m.clone(), v.clone(), loss.clone()))
    for a, b in zip(*runs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
@pytest.mark.parametrize("t", [1, 7])
def test_adam_single_step_well_conditioned_entries(algo, t):
    """One update at step number t (t = 7 without the six before it: the device
    counter is resynchronised), both update paths."""
    st = _st()
    prob = synth.make_deconv(2, E=4)
    d, w, rng = _data(prob, seed=6)
    p0 = synth.eval_point(prob, "near", rng)
    lrv = prob.lr_vector()
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    plan = _plan(prob, d, w, algo=algo)
    x = torch.tensor(p0, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(x)
    v = torch.zeros_like(x)
    plan.step(x, m, v, t, lr4)
    po = p0.copy()
    _, go = ora.loss_grad(prob, d, w, po)
    mo, vo = np.zeros_like(po), np.zeros_like(po)
    ora.adam_step(po, go, mo, vo, t, lrv)
    good = np.abs(go) > 1e-3 * np.abs(go).max()
    xf = x.cpu().numpy().astype(np.float64)
    err = np.abs(xf - po)[good] / np.maximum(np.abs(po[good]), lrv[good])
    _say(f"adam single step: {good.sum()} entries, max rel err {err.max():.2e}")
    assert err.max() <= 1e-5
    np.testing.assert_allclose(m.cpu().numpy()[good], mo[good], rtol=1e-3)


def test_loss_grad_before_set_frames_is_an_error():
    st = _st()
    prob = synth.make_deconv(1)
    plan = st.Plan.for_problem(prob)
    with pytest.raises(st.StarredError) as e:
        plan.loss_grad(prob.params_true)
    assert e.value.code == st.ESTATE


# --------------------------------------------------------------------------- #
# PSF-reconstruction mode (Eqs. 2-7)                                           #
# --------------------------------------------------------------------------- #

PSF_CASES = [
    ("psf_small_s3", dict(S=4, n=16, s=3, J=4)),
    ("psf_s2", dict(S=5, n=24, s=2, J=4)),
    # ragged data tiles (37 = 4 x 8 + 5 rows, 32 + 5 columns) and grid tiles (111)
    ("psf_s3_ragged", dict(S=3, n=37, s=3, J=4)),
    # s = 1: more stars than one adjoint batch holds, ragged 21 x 21 grid
    ("psf_s1_batches", dict(S=12, n=21, s=1, J=3)),
    # a 384 x 384 grid: the tiles are the same size at any grid (no per-star planes in LDS)
    ("psf_n128_s3", dict(S=2, n=128, s=3, J=5)),
    ("psf_cfg3", dict()),
]


def _psf_setup(kw, seed):
    st = _st()
    prob = synth.make_psf(**kw)
    rng = np.random.default_rng(seed)
    m = ora.psf_model(prob, prob.params_true)
    d, w = synth.add_noise(m, rng, sigma_bg=prob.sigma_bg, poisson=False)
    plan = st.Plan.for_psf(prob)
    plan.set_frames(d, w, None, prob.W)
    return prob, d, w, rng, plan


@pytest.mark.parametrize("name,kw", PSF_CASES, ids=[c[0] for c in PSF_CASES])
def test_psf_render_and_model(name, kw):
    prob, d, w, rng, plan = _psf_setup(kw, 41)
    p = synth.psf_eval_point(prob, "near", rng)
    s_dev = plan.render_scene(p).cpu().numpy()
    s_ora = ora.psf_render(prob.N, p)
    assert np.abs(s_dev - s_ora).max() <= 2e-6 * np.abs(s_ora).max()
    m_dev = plan.psf_model(p).cpu().numpy()
    m_ora = ora.psf_model(prob, p)
    _check_frames(m_dev, m_ora, [prob.n] * prob.S, 2e-6)


@pytest.mark.parametrize("name,kw", PSF_CASES, ids=[c[0] for c in PSF_CASES])
@pytest.mark.parametrize("point", ["init", "near"])
def test_psf_loss_grad_parity(name, kw, point):
    prob, d, w, rng, plan = _psf_setup(kw, 42)
    p = synth.psf_eval_point(prob, point, rng)
    loss, grad = plan.loss_grad(p)
    loss = loss.cpu().numpy()
    grad = grad.cpu().numpy().astype(np.float64)
    NN = prob.N * prob.N
    alpha_dev = plan.starlet_fwd(p[5:5 + NN]).cpu().numpy()
    so, nsub = parity.tie_override(prob.N, prob.J, p[5:5 + NN], alpha_dev)
    lo, go = ora.psf_loss_grad(prob, d, w, p, sgn_override=so)
    rl = abs(loss[2] - lo[2]) / abs(lo[2])
    blocks = {k: parity.rel_err(parity.psf_blocks(prob, grad)[k], v)
              for k, v in parity.psf_blocks(prob, go).items()}
    _say(f"{name}/{point}: loss rel {rl:.2e}; grad {blocks}; ties {nsub}")
    assert rl <= 1e-6
    assert parity.rel_err(grad, go) <= 1e-4
    for k, v in blocks.items():
        assert v <= 1e-4, (k, v)


def test_psf_line_search_evaluations_forward_only():
    prob, d, w, rng, plan = _psf_setup(dict(S=4, n=16, s=3, J=4), 43)
    p = synth.psf_eval_point(prob, "init", rng)
    _, g = plan.loss_grad(p)
    g = g.cpu().numpy().astype(np.float64)
    # Armijo backtracking along the negative gradient with forward-only evaluations
    f0 = plan.loss_grad(p, want_grad=False)[0][2].item()
    step = 1.0 / max(np.abs(g).max(), 1e-30)
    for _ in range(30):
        trial = synth.f32(p - step * g)
        f1 = plan.loss_grad(trial, want_grad=False)[0][2].item()
        lo, _ = ora.psf_loss_grad(prob, d, w, trial, want_grad=False)
        assert abs(f1 - lo[2]) <= 1e-6 * abs(lo[2])
        if f1 <= f0 - 1e-4 * step * float(np.dot(g, g)):
            break
        step *= 0.5
    assert f1 < f0


# --------------------------------------------------------------------------- #
# The plain per-epoch baseline computes the same loss and gradient             #
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("name,make", [LG_CASES[0], LG_CASES[1], LG_CASES[3]],
                         ids=[LG_CASES[i][0] for i in (0, 1, 3)])
def test_plain_baseline_parity(name, make):
    prob = make()
    d, w, rng = _data(prob, seed=7)
    plan = _plan(prob, d, w, 1)
    p = synth.eval_point(prob, "near", rng)
    loss, grad = plan.loss_grad_plain(p)
    loss = loss.cpu().numpy()
    grad = grad.cpu().numpy().astype(np.float64)
    NN = prob.N * prob.N
    so, _ = parity.tie_override(prob.N, prob.J, p[:NN], plan.starlet_fwd(p[:NN]).cpu().numpy())
    lo, go = ora.loss_grad(prob, d, w, p, sgn_override=so)
    rl = abs(loss[2] - lo[2]) / abs(lo[2])
    rg = parity.rel_err(grad, go)
    _say(f"plain {name}: loss rel {rl:.2e} grad rel {rg:.2e}")
    assert rl <= 1e-6 and rg <= 1e-4


# --------------------------------------------------------------------------- #
# Graph mode: every replay equals the eager result                             #
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_graph_replays_match_eager(algo):
    st = _st()
    prob = synth.make_deconv(2, E=8)
    d, w, rng = _data(prob, seed=8)
    p = torch.tensor(synth.eval_point(prob, "near", rng), dtype=torch.float32, device="cuda")
    plan = _plan(prob, d, w, algo)
    le, ge = plan.loss_grad(p)
    le, ge = le.clone(), ge.clone()
    plan.set_graph_mode(True)
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty(prob.n_params, dtype=torch.float32, device="cuda")
    for rep in range(4):
        loss.fill_(-1.0)
        grad.fill_(-1.0)
        plan.loss_grad(p, grad_out=grad, loss_out=loss)
        torch.cuda.synchronize()
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()  # eager work between replays
        assert torch.equal(loss, le), rep
        assert torch.equal(grad, ge), rep
    # optimiser steps: graph replays vs eager steps from the same state
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    xg, xe = p.clone(), p.clone()
    mg, vg = torch.zeros_like(p), torch.zeros_like(p)
    me, ve = torch.zeros_like(p), torch.zeros_like(p)
    plan2 = _plan(prob, d, w, algo)
    for t in range(1, 6):
        plan.step(xg, mg, vg, t, lr4, loss_out=loss)
        plan2.step(xe, me, ve, t, lr4)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe), t
        assert torch.equal(mg, me) and torch.equal(vg, ve), t


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_graph_replay_after_rebinding_frames(algo):
    """A captured graph holds the bound data pointers: after set_frames with new data
    (new device arrays), a replay must read the new data, as an eager call does."""
    st = _st()
    prob = synth.make_deconv(2, E=6)
    d, w, rng = _data(prob, seed=18)
    p = torch.tensor(synth.eval_point(prob, "near", rng), dtype=torch.float32, device="cuda")
    plan = _plan(prob, d, w, algo)
    plan.set_graph_mode(True)
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty(prob.n_params, dtype=torch.float32, device="cuda")
    plan.loss_grad(p, grad_out=grad, loss_out=loss)  # captured with the first data
    torch.cuda.synchronize()
    l_first = loss.clone()
    d2 = synth.f32(d + rng.normal(0.0, 30.0, d.shape))
    plan.set_frames(d2, w, prob.kernels, prob.W)
    _ = (torch.randn(1000, device="cuda") * 2).sum().item()  # the old arrays' memory gets reused
    plan.loss_grad(p, grad_out=grad, loss_out=loss)
    torch.cuda.synchronize()
    eager = _plan(prob, d2, w, algo)
    le, ge = eager.loss_grad(p)
    torch.cuda.synchronize()
    assert not torch.equal(loss, l_first)
    assert torch.equal(loss, le) and torch.equal(grad, ge)


def test_graph_mode_psf():
    prob, d, w, rng, plan = _psf_setup(dict(S=4, n=16, s=3, J=4), 44)
    p = torch.tensor(synth.psf_eval_point(prob, "near", rng), dtype=torch.float32, device="cuda")
    le, ge = plan.loss_grad(p)
    le, ge = le.clone(), ge.clone()
    plan.set_graph_mode(True)
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty(prob.n_params, dtype=torch.float32, device="cuda")
    for rep in range(3):
        grad.fill_(0.0)
        plan.loss_grad(p, grad_out=grad, loss_out=loss)
        torch.cuda.synchronize()
        assert torch.equal(loss, le) and torch.equal(grad, ge), rep


def test_psf_adam_steps_match_oracle():
    """PSF-mode Adam steps: the update adds the prior's gradient to dchi/db itself
    (the adjoint runs beside the starlet branch), so four steps are checked against
    the oracle's Adam on the oracle's whole gradient, and graph steps against eager ones."""
    st = _st()
    prob, d, w, rng, plan = _psf_setup(dict(S=4, n=16, s=3, J=4), 45)
    p0 = synth.psf_eval_point(prob, "near", rng)
    NN = prob.N * prob.N
    lr4 = [1e-4, 1e-7, 1e-4 * float(np.median(prob.a)), 1e-3]
    lrv = np.concatenate([np.full(5, lr4[0]), np.full(NN, lr4[1]), np.full(prob.S, lr4[2]),
                          np.full(2 * prob.S, lr4[3])])
    x = torch.tensor(p0, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(x)
    v = torch.zeros_like(x)
    po = p0.astype(np.float64)
    mo, vo = np.zeros_like(po), np.zeros_like(po)
    # the first Adam step moves each entry by lr sign(g); later ones weigh magnitudes,
    # so a missing or doubled prior term in dchi/db shows by the fourth
    for t in range(1, 5):
        plan.step(x, m, v, t, lr4)
        alpha_dev = plan.starlet_fwd(synth.f32(po[5:5 + NN])).cpu().numpy()
        so, _ = parity.tie_override(prob.N, prob.J, po[5:5 + NN], alpha_dev)
        _, go = ora.psf_loss_grad(prob, d, w, po, sgn_override=so)
        ora.adam_step(po, go, mo, vo, t, lrv)
    good = np.abs(vo) > 1e-6 * np.abs(vo).max()
    xf = x.cpu().numpy().astype(np.float64)
    err = np.abs(xf - po)[good] / np.maximum(np.abs(po[good]), lrv[good])
    _say(f"psf adam 4 steps: {good.sum()} entries, max rel err {err.max():.2e}")
    assert err.max() <= 1e-4
    # eager and graph steps agree bit for bit
    xe, me, ve = x.clone(), m.clone(), v.clone()
    xg, mg, vg = x.clone(), m.clone(), v.clone()
    le = torch.empty(3, dtype=torch.float64, device="cuda")
    lg = torch.empty(3, dtype=torch.float64, device="cuda")
    for t in range(2, 12):
        plan.step(xe, me, ve, t, lr4, loss_out=le)
    plan.set_graph_mode(True)
    plan.steps(xg, mg, vg, 2, lr4, 10, loss_out=lg)
    plan.set_graph_mode(False)
    torch.cuda.synchronize()
    assert torch.equal(xg, xe) and torch.equal(mg, me) and torch.equal(vg, ve) and torch.equal(lg, le)


# --------------------------------------------------------------------------- #
# Supernova (ragged) and crowded-field workloads                               #
# --------------------------------------------------------------------------- #

BIG_CASES = [
    # every stamp size of the supernova workload, 10 epochs
    ("cfg4_sizes", lambda: synth.make_deconv(4, E=10)),
    # crowded field shape with 30 sources and 8 scales, 2 epochs at half the side
    ("cfg5_shape", lambda: _cfg5_half(2)),
]


def _cfg5_half(E):
    prob = synth.make_deconv(5, E=E)
    # same kernels, sources and scales on a 128^2-data (256^2-grid) crop of the field
    N = 256
    h = prob.h.reshape(512, 512)[128:384, 128:384]
    c = prob.c.reshape(-1, 2) - 128.0
    c = np.clip(c, 8, N - 9)
    return synth.DeconvProblem(**{**prob.__dict__, "n": np.full(E, 128, np.int32), "N": N,
                                  "h": synth.f32(h).ravel(), "c": synth.f32(c).ravel()})


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
@pytest.mark.parametrize("name,make", BIG_CASES, ids=[c[0] for c in BIG_CASES])
def test_loss_grad_parity_large_shapes(name, make, algo):
    prob = make()
    d, w, rng = _data(prob, seed=9)
    plan = _plan(prob, d, w, algo)
    p = synth.eval_point(prob, "near", rng)
    _compare_loss_grad(prob, d, w, p, plan, f"{name}/{ALGO_ID[algo]}")


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_cfg4_full_size_sampled_frames_and_properties(algo):
    """1000 ragged epochs in one plan: per-frame model parity on one frame of each
    stamp size, the adjoint identity and exact central differences at full size."""
    st = _st()
    prob = synth.make_deconv(4)
    rng = np.random.default_rng(10)
    scene = synth.f32(rng.standard_normal(prob.fine_size) * 50)
    plan = st.Plan.for_problem(prob, conv_algo=algo)
    plan.set_frames(np.zeros(prob.data_size), np.ones(prob.data_size), prob.kernels, prob.W)
    model = plan.convolve_subsample(scene).cpu().numpy().astype(np.float64)
    offs_d = np.concatenate([[0], np.cumsum(prob.n.astype(np.int64) ** 2)])
    offs_f = np.concatenate([[0], np.cumsum((prob.s * prob.n.astype(np.int64)) ** 2)])
    offs_k = np.concatenate([[0], np.cumsum(prob.K.astype(np.int64) ** 2)])
    for side in sorted(set(prob.n.tolist())):
        i = int(np.nonzero(prob.n == side)[0][0])
        ref = ora.conv_sub([side], [prob.K[i]], prob.s, prob.kernels[offs_k[i]:offs_k[i + 1]],
                           scene[offs_f[i]:offs_f[i + 1]])
        got = model[offs_d[i]:offs_d[i + 1]]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        _say(f"cfg4 full frame {i} (n={side}): max rel err {err:.2e}")
        assert err <= 1e-5
    resid = synth.f32(rng.standard_normal(prob.data_size))
    adj = plan.convolve_subsample_adj(resid).cpu().numpy().astype(np.float64)
    lhs, rhs = np.dot(model, resid), np.dot(scene, adj)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(model) * np.linalg.norm(resid)
    # loss + gradient at full size: chi^2 is quadratic in h, so central differences are exact
    d = synth.f32(model + rng.normal(0, 10, model.shape))
    w = np.full(prob.data_size, 0.01)
    plan.set_frames(d, w, prob.kernels, prob.W)
    plan0 = st.Plan.for_problem(prob, conv_algo=algo, lam=0.0)
    plan0.set_frames(d, w, prob.kernels, prob.W)
    p = synth.eval_point(prob, "near", rng)
    _, g = plan0.loss_grad(p)
    g = g.cpu().numpy().astype(np.float64)
    NN = prob.N ** 2
    delta = np.zeros(prob.n_params)
    delta[:NN] = rng.standard_normal(NN)
    pp, pm = synth.f32(p + delta), synth.f32(p - delta)
    fd = plan0.loss_grad(pp, want_grad=False)[0][2].item() - plan0.loss_grad(pm, want_grad=False)[0][2].item()
    an = float(np.dot(g, pp - pm))
    _say(f"cfg4 full: directional difference {fd:.8e} vs gradient {an:.8e}")
    assert abs(fd - an) <= 1e-4 * abs(an)


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_cfg5_full_size_sampled_frame_and_properties(algo):
    """The large field at full size (12 epochs of 256^2 data, 512^2 grid, 128^2 kernels,
    30 sources, 8 scales): model parity on one whole frame, the adjoint identity, and
    exact central differences of the loss along h (chi^2 is quadratic in h)."""
    st = _st()
    prob = synth.make_deconv(5)
    rng = np.random.default_rng(12)
    scene = synth.f32(rng.standard_normal(prob.fine_size) * 50)
    plan = st.Plan.for_problem(prob, conv_algo=algo)
    plan.set_frames(np.zeros(prob.data_size), np.ones(prob.data_size), prob.kernels, prob.W)
    model = plan.convolve_subsample(scene).cpu().numpy().astype(np.float64)
    n0, K0, F0 = int(prob.n[0]), int(prob.K[0]), prob.s * int(prob.n[0])
    i = prob.E - 1  # the last frame
    ref = ora.conv_sub([n0], [K0], prob.s, prob.kernels[i * K0 * K0:(i + 1) * K0 * K0],
                       scene[i * F0 * F0:(i + 1) * F0 * F0])
    got = model[i * n0 * n0:(i + 1) * n0 * n0]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _say(f"cfg5 full frame {i}: max rel err {err:.2e}")
    assert err <= 1e-5
    resid = synth.f32(rng.standard_normal(prob.data_size))
    adj = plan.convolve_subsample_adj(resid).cpu().numpy().astype(np.float64)
    lhs, rhs = np.dot(model, resid), np.dot(scene, adj)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(model) * np.linalg.norm(resid)
    d = synth.f32(model + rng.normal(0, 10, model.shape))
    w = np.full(prob.data_size, 0.01)
    plan0 = st.Plan.for_problem(prob, conv_algo=algo, lam=0.0)
    plan0.set_frames(d, w, prob.kernels, prob.W)
    p = synth.eval_point(prob, "near", rng)
    _, g = plan0.loss_grad(p)
    g = g.cpu().numpy().astype(np.float64)
    NN = prob.N ** 2
    delta = np.zeros(prob.n_params)
    # a long step: the difference is exact at any length (quadratic), and the FP32
    # rounding of the two losses (~1 at this size) must stay far below it
    delta[:NN] = 30.0 * rng.standard_normal(NN)
    pp, pm = synth.f32(p + delta), synth.f32(p - delta)
    fd = plan0.loss_grad(pp, want_grad=False)[0][2].item() - plan0.loss_grad(pm, want_grad=False)[0][2].item()
    an = float(np.dot(g, pp - pm))
    _say(f"cfg5 full: directional difference {fd:.8e} vs gradient {an:.8e}")
    assert abs(fd - an) <= 1e-4 * abs(an)


# --------------------------------------------------------------------------- #
# Noise propagation to the starlet coefficients (Sec. 2.3, App. B)             #
# --------------------------------------------------------------------------- #

def _noise_case():
    # cfg1 shapes: frame 0 of 32^2 data, s = 2, 64^2 kernel, 64^2 grid, J = 3
    prob = synth.make_deconv(1)
    d, w, rng = _data(prob, seed=31)
    plan = _plan(prob, d, w, algo=2)
    n0, K0 = int(prob.n[0]), int(prob.K[0])
    k0 = np.asarray(prob.kernels[:K0 * K0], np.float64)
    sig2 = 1.0 / np.asarray(w[:n0 * n0], np.float64)  # the frame's own noise map
    return prob, plan, n0, K0, k0, sig2


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("per_pixel", [True, False], ids=["per_pixel", "per_scale"])
def test_noise_weights_with_given_draws_match_oracle(per_pixel):
    """Caller-supplied normal draws: the device pipeline (weighting, S^T through an s = 1
    FFT plan, embedding, batched starlet, FP64 moments) against the oracle's Monte Carlo
    on the same draws; 40 realizations = one full and one partial batch."""
    prob, plan, n0, K0, k0, sig2 = _noise_case()
    R = 40
    F = prob.s * n0
    z = np.random.default_rng(32).standard_normal((R, F * F)).astype(np.float32)
    got = plan.noise_weights(sig2, R, normals=z, per_pixel=per_pixel).cpu().numpy()
    ref = ora.noise_weights_mc(n0, K0, prob.s, prob.N, prob.J, k0, sig2, R, normals=z.astype(np.float64),
                               per_pixel=per_pixel)
    err = _rel(got, ref)
    _say(f"noise W given draws ({'pixel' if per_pixel else 'scale'}): rel err {err:.2e}")
    assert err <= 1e-4


def test_noise_weights_device_philox_draws_match_oracle_generator():
    """Device-drawn noise (Philox4x32-10 + Box-Muller on the GPU) against the oracle's
    own implementation of the same generator: the same draws, hence the same W."""
    prob, plan, n0, K0, k0, sig2 = _noise_case()
    R, seed = 40, 0xC0FFEE1234
    got = plan.noise_weights(sig2, R, seed=seed).cpu().numpy()
    ref = ora.noise_weights_mc(n0, K0, prob.s, prob.N, prob.J, k0, sig2, R, seed=seed, per_pixel=True)
    err = _rel(got, ref)
    _say(f"noise W device Philox: rel err {err:.2e}")
    assert err <= 1e-4
    again = plan.noise_weights(sig2, R, seed=seed).cpu().numpy()
    assert np.array_equal(got, again)
    other = plan.noise_weights(sig2, R, seed=seed + 1).cpu().numpy()
    assert not np.array_equal(got, other)


def test_noise_weights_converge_to_exact_variance():
    """Many device realizations against the exact variance of the propagated noise
    (sum over fine pixels of squared impulse responses): median relative error of W^2
    within 4 standard errors of a variance estimate from R draws."""
    st = _st()
    prob = synth.make_small_deconv(107, 2, [12, 12], [9, 9], 2, 32, 1, 4)
    d, w, rng = _data(prob, seed=33)
    plan = _plan(prob, d, w, algo=2)
    n0, K0 = int(prob.n[0]), int(prob.K[0])
    k0 = np.asarray(prob.kernels[:K0 * K0], np.float64)
    sig2 = np.random.default_rng(34).uniform(1.0, 4.0, n0 * n0)
    R = 4000
    Wd = plan.noise_weights(sig2, R, seed=7).cpu().numpy().reshape(prob.J, prob.N, prob.N).astype(np.float64)
    var = ora.noise_variance(n0, K0, prob.s, prob.N, prob.J, k0, sig2).reshape(prob.J, prob.N, prob.N)
    inside = var > 1e-10 * var.max()
    rel = np.abs(Wd[inside] ** 2 - var[inside]) / var[inside]
    _say(f"noise W vs exact variance: median rel {np.median(rel):.3e} (bound {4 * np.sqrt(2 / R):.3e})")
    assert np.median(rel) < 4 * np.sqrt(2.0 / R)


def test_noise_weights_argument_errors():
    st = _st()
    prob, plan, n0, K0, k0, sig2 = _noise_case()
    with pytest.raises(st.StarredError):
        plan.noise_weights(sig2, 1)
    with pytest.raises(st.StarredError):
        plan.noise_weights(sig2, 10, frame=prob.E)


# --------------------------------------------------------------------------- #
# Point-source prior (Eq. 11, third term) and its App. C estimate              #
# --------------------------------------------------------------------------- #

def _compare_with_pts(prob, d, w, p, plan, lam_pts, label, plain=False):
    NN = prob.N * prob.N
    if plain:
        loss, grad = plan.loss_grad_plain(p)
    else:
        loss, grad = plan.loss_grad(p)
    loss = loss.cpu().numpy()
    grad = grad.cpu().numpy().astype(np.float64)
    so_h, n1 = parity.tie_override(prob.N, prob.J, p[:NN], plan.starlet_fwd(p[:NN]).cpu().numpy())
    alpha_P = plan.starlet_fwd(plan.pts_image(p)).cpu().numpy()
    so_P, n2 = parity.tie_override(prob.N, prob.J, ora.pts_image(prob, p), alpha_P)
    lo, go = ora.loss_grad(prob, d, w, p, sgn_override=so_h, lam_pts=lam_pts, sgn_override_pts=so_P)
    rl = abs(loss[2] - lo[2]) / abs(lo[2])
    blocks = {k: parity.rel_err(parity.deconv_blocks(prob, grad)[k], v)
              for k, v in parity.deconv_blocks(prob, go).items() if np.linalg.norm(v) > 0}
    _say(f"{label}: loss rel {rl:.2e} (l1 {abs(loss[1]-lo[1])/abs(lo[1]):.2e}); grad {blocks}; ties {n1}+{n2}")
    assert rl <= 1e-6
    assert parity.rel_err(grad, go) <= 1e-4
    for k, v in blocks.items():
        assert v <= 1e-4, (k, v)


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
@pytest.mark.parametrize("name,make", [LG_CASES[0], LG_CASES[1], LG_CASES[3]], ids=["cfg1", "cfg2_E6", "small_s3"])
def test_loss_grad_with_point_source_prior(name, make, algo):
    prob = make()
    d, w, rng = _data(prob, seed=41)
    plan = _plan(prob, d, w, algo=algo)
    p = synth.eval_point(prob, "near", rng)
    lam_pts = 0.6 * prob.lam
    plan.set_lambda_pts(lam_pts)
    _compare_with_pts(prob, d, w, p, plan, lam_pts, f"{name}/{ALGO_ID[algo]}/pts")
    # graph replay of the same evaluation
    plan.set_graph_mode(True)
    _compare_with_pts(prob, d, w, p, plan, lam_pts, f"{name}/{ALGO_ID[algo]}/pts graph")
    plan.set_graph_mode(False)
    # and off again: back to the two-term loss
    plan.set_lambda_pts(0.0)
    _compare_loss_grad(prob, d, w, p, plan, f"{name}/{ALGO_ID[algo]}/pts off")


def test_plain_baseline_with_point_source_prior():
    prob = synth.make_deconv(2, E=6)
    d, w, rng = _data(prob, seed=42)
    plan = _plan(prob, d, w)
    p = synth.eval_point(prob, "near", rng)
    plan.set_lambda_pts(1.3)
    _compare_with_pts(prob, d, w, p, plan, 1.3, "plain/pts", plain=True)


@pytest.mark.parametrize("name,make", [LG_CASES[0], LG_CASES[1]], ids=["cfg1", "cfg2_E6"])
def test_lambda_pts_estimate_matches_oracle(name, make):
    prob = make()
    d, w, rng = _data(prob, seed=43)
    plan = _plan(prob, d, w)
    for point in ("init", "near"):
        p = synth.eval_point(prob, point, rng)
        got = plan.estimate_lambda_pts(p)
        ref = ora.lambda_pts_estimate(prob, p)
        _say(f"{name}/{point}: lambda_pts estimate {got:.6g} oracle {ref:.6g}")
        assert got == pytest.approx(ref, rel=1e-4)


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_adabelief_steps_against_oracle(algo):
    """The AdaBelief rule (the optimiser of the paper's fits) through the same step: a
    single step on well-conditioned entries, then 50 steps against the oracle's
    trajectory (graph mode, so the rule is part of the captured update)."""
    st = _st()
    prob = synth.make_deconv(1)
    d, w, rng = _data(prob, seed=44)
    p0 = synth.eval_point(prob, "near", rng)
    lrv = prob.lr_vector()
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    plan = _plan(prob, d, w, algo=algo)
    x = torch.tensor(p0, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(x)
    v = torch.zeros_like(x)
    kw = dict(rule=st.ADABELIEF, eps=1e-16, eps_root=1e-16)
    plan.step(x, m, v, 1, lr4, **kw)
    po = p0.copy()
    mo, vo = np.zeros_like(po), np.zeros_like(po)
    _, go = ora.loss_grad(prob, d, w, po)
    ora.adabelief_step(po, go, mo, vo, 1, lrv, eps=1e-16, eps_root=1e-16)
    good = np.abs(go) > 1e-3 * np.abs(go).max()
    xf = x.cpu().numpy().astype(np.float64)
    err = np.abs(xf - po)[good] / np.maximum(np.abs(po[good]), lrv[good])
    _say(f"adabelief single step: {good.sum()} entries, max rel err {err.max():.2e}")
    assert err.max() <= 1e-5
    plan.set_graph_mode(True)
    NN = prob.N ** 2
    for t in range(2, 51):
        plan.step(x, m, v, t, lr4, **kw)
        so, _ = parity.tie_override(prob.N, prob.J, po[:NN], plan.starlet_fwd(po[:NN]).cpu().numpy())
        _, go = ora.loss_grad(prob, d, w, po, sgn_override=so)
        ora.adabelief_step(po, go, mo, vo, t, lrv, eps=1e-16, eps_root=1e-16)
    plan.set_graph_mode(False)
    lg = plan.loss_grad(x)[0].cpu().numpy()
    lo, _ = ora.loss_grad(prob, d, w, po, want_grad=False)
    cdev = x.cpu().numpy().astype(np.float64)[-2 * prob.M:]
    _say(f"adabelief 50: loss dev {lg[2]:.6e} oracle {lo[2]:.6e} rel {abs(lg[2] - lo[2]) / abs(lo[2]):.2e}; "
         f"c dev {cdev} oracle {po[-2 * prob.M:]}")
    assert abs(lg[2] - lo[2]) / abs(lo[2]) <= 1e-4
    assert np.abs(cdev - po[-2 * prob.M:]).max() <= 0.01


# --------------------------------------------------------------------------- #
# L-BFGS                                                                       #
# --------------------------------------------------------------------------- #

def test_lbfgs_direction_matches_oracle_two_loop():
    """The device two-loop recursion against the oracle's, on gradient-difference
    pairs of the real loss (a wrapped ring of 7 pairs in 5 slots)."""
    prob = synth.make_deconv(1)
    d, w, rng = _data(prob, seed=45)
    plan = _plan(prob, d, w)
    n = prob.n_params
    m = 5
    S = np.zeros((m, n), np.float32)
    Y = np.zeros((m, n), np.float32)
    p = synth.eval_point(prob, "near", rng)
    _, g0 = ora.loss_grad(prob, d, w, p, lam=0.0)
    newest = -1
    for k in range(7):
        s = synth.f32(1e-2 * rng.standard_normal(n) * np.maximum(np.abs(p), 1.0))
        _, g1 = ora.loss_grad(prob, d, w, synth.f32(p + s), lam=0.0)
        newest = (newest + 1) % m
        S[newest], Y[newest] = s, synth.f32(g1 - g0)
    g = synth.f32(g0)
    for count in (0, 1, 3, 5):
        got = plan.lbfgs_direction(g, S, Y, count, newest).cpu().numpy()
        ref = ora.lbfgs_direction(g, S, Y, count, newest)
        err = parity.rel_err(got, ref)
        _say(f"lbfgs direction count {count}: rel err {err:.2e}")
        assert err <= 1e-4


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
def test_lbfgs_iterations_decrease_the_loss(algo):
    """Iterations never raise the loss, reach scipy's L-BFGS-B on the oracle (same
    start, same history length, 30 iterations, lambda = 0) to 1e-3, and the reported
    loss is the loss at the returned point."""
    st = _st()
    prob = synth.make_deconv(1)
    d, w, rng = _data(prob, seed=46)
    plan = st.Plan.for_problem(prob, conv_algo=algo, lam=0.0)
    plan.set_frames(d, w, prob.kernels, prob.W)
    x0 = synth.eval_point(prob, "init", rng)
    x = torch.tensor(x0, dtype=torch.float32, device="cuda")
    l0 = plan.loss_grad(x)[0][2].item()
    opt = plan.lbfgs(m=8)
    losses = []
    for _ in range(6):
        f, ev = opt.run(x, 5)
        losses.append(f)
    _say(f"lbfgs {ALGO_ID[algo]}: start {l0:.6e}, after 5..30 iterations {['%.6e' % v for v in losses]}")
    assert all(b <= a * (1 + 1e-12) for a, b in zip([l0] + losses, losses))
    import scipy.optimize
    res = scipy.optimize.minimize(lambda q: (lambda lg: (lg[0][2], lg[1]))(ora.loss_grad(prob, d, w, q, lam=0.0)),
                                  x0, jac=True, method="L-BFGS-B", options=dict(maxiter=30, maxcor=8))
    _say(f"scipy L-BFGS-B on the oracle, 30 iterations: {res.fun:.6e}")
    assert losses[-1] <= (1 + 1e-3) * res.fun
    assert plan.loss_grad(x)[0][2].item() == pytest.approx(losses[-1], rel=1e-6)


def test_lbfgs_box_bounds_hold():
    st = _st()
    prob = synth.make_deconv(1)
    d, w, rng = _data(prob, seed=47)
    plan = _plan(prob, d, w)
    x0 = synth.eval_point(prob, "near", rng)
    n, NN, E, M = prob.n_params, prob.N ** 2, prob.E, prob.M
    lo = np.full(n, -np.inf, np.float32)
    hi = np.full(n, np.inf, np.float32)
    lo[:NN] = 0.0                                  # non-negative h
    c0 = x0[NN + E + E * M:]
    lo[NN + E + E * M:] = c0 - 0.05                # positions within 0.05 px
    hi[NN + E + E * M:] = c0 + 0.05
    x = torch.tensor(np.clip(x0, lo, hi), dtype=torch.float32, device="cuda")
    opt = plan.lbfgs(m=6, lo=lo, hi=hi)
    f, ev = opt.run(x, 15)
    xf = x.cpu().numpy()
    _say(f"lbfgs with bounds: loss {f:.6e} after {ev} evaluations")
    assert np.all(xf >= lo) and np.all(xf <= hi)


def test_lbfgs_psf_mode():
    """The paper's PSF fits use L-BFGS: iterations on the PSF-mode loss decrease it."""
    prob, d, w, rng, plan = _psf_setup(PSF_CASES[1][1], 48)
    x = torch.tensor(synth.psf_eval_point(prob, "near", rng), dtype=torch.float32, device="cuda")
    l0 = plan.loss_grad(x)[0][2].item()
    f, ev = plan.lbfgs(m=6).run(x, 20)
    _say(f"lbfgs psf: {l0:.6e} -> {f:.6e} in {ev} evaluations")
    assert f < l0


def test_pipeline_psf_fits_then_joint_deconvolution():
    """The paper's two-stage workflow (f3's pipeline): per-epoch PSF reconstruction
    from star stamps (PSF mode, L-BFGS), the fitted narrow PSFs s_i rendered on the
    device (starred_render_scene) as the deconvolution kernels, then the joint
    deconvolution (Adam steps, starred_steps). The data are made with the true
    PSFs; the fit with the reconstructed kernels must land close to the one with
    the true kernels."""
    st = _st()
    E, s, n_star, M, J = 3, 2, 16, 2, 3
    K = s * n_star
    kern_true, kern_fit = [], []
    for e in range(E):
        pp = synth.make_psf(cfg=3, rep=e, S=6, n=n_star, s=s, J=3)
        rng = np.random.default_rng(300 + e)
        d, w = synth.add_noise(ora.psf_model(pp, pp.params_true), rng, sigma_bg=pp.sigma_bg, poisson=False)
        plan = st.Plan.for_psf(pp)
        plan.set_frames(d, w, None, pp.W)
        NN = pp.N ** 2
        # a start as from the data: Moffat within a few per cent, amplitudes within 5 %,
        # positions within 0.2 px, no pixel grid
        x0 = synth.psf_eval_point(pp, "near", rng)
        x0[5:5 + NN] = 0.0
        truth = torch.tensor(pp.params_true, dtype=torch.float32, device="cuda")
        ft = plan.loss_grad(truth)[0][2].item()
        kern_true.append(plan.render_scene(truth).cpu().numpy().astype(np.float64))
        # stage 1: the Moffat, amplitudes and positions by L-BFGS with the pixel grid
        # b held at zero (a box with lo = hi there; A, widths > 0, beta > 1, a >= 0)
        lo = np.full(pp.n_params, -np.inf, np.float32)
        hi = np.full(pp.n_params, np.inf, np.float32)
        lo[[0, 1, 2]] = 1e-6
        lo[4], hi[4] = 1.05, 20.0
        lo[5:5 + NN] = hi[5:5 + NN] = 0.0
        lo[5 + NN:5 + NN + pp.S] = 0.0
        x = torch.tensor(np.clip(x0, lo, hi), dtype=torch.float32, device="cuda")
        f0 = plan.loss_grad(x)[0][2].item()
        f1, ev = plan.lbfgs(m=10, lo=lo, hi=hi).run(x, 100)
        err1 = np.abs(plan.render_scene(x).cpu().numpy() - kern_true[-1]).sum() / np.abs(kern_true[-1]).sum()
        # stage 2: everything, b included, by AdaBelief steps (per-block rates)
        m = torch.zeros_like(x)
        v = torch.zeros_like(x)
        lr4 = [1e-4, 1e-7, 1e-4 * float(np.median(pp.a)), 1e-3]
        f2 = plan.steps(x, m, v, 1, lr4, 600, rule=st.ADABELIEF, eps=1e-16, eps_root=1e-16)[2].item()
        kern_fit.append(plan.render_scene(x).cpu().numpy().astype(np.float64))
        err = np.abs(kern_fit[-1] - kern_true[-1]).sum() / np.abs(kern_true[-1]).sum()
        _say(f"pipeline psf {e}: loss {f0:.4e} -> {f1:.4e} (L-BFGS, {ev} evals, kernel L1 error {err1:.2e}) "
             f"-> {f2:.4e} (AdaBelief; at the truth {ft:.4e}), kernel L1 error {err:.2e}")
        # (measured: L-BFGS kernels within 0.06-0.075 in L1, after AdaBelief 0.05-0.11)
        assert f1 < f0 and f2 < f1 and err1 < 0.12 and err < 0.16
    dp = synth.make_small_deconv(311, E, [n_star], [K], s, K, M, J)
    dp.kernels = synth.f32(np.concatenate([k.ravel() for k in kern_true]))
    d, w, rng = _data(dp, seed=312)  # the data: true kernels
    p0 = synth.eval_point(dp, "init", rng)
    lr4 = [0.5, 0.05, 20.0, 0.01]  # the workloads' Adam rates for h, Gamma, a, c
    fits = []
    for kern in (kern_true, kern_fit):
        plan = st.Plan.for_problem(dp)
        plan.set_frames(d, w, synth.f32(np.concatenate([k.ravel() for k in kern])), dp.W)
        x = torch.tensor(p0, dtype=torch.float32, device="cuda")
        m = torch.zeros_like(x)
        v = torch.zeros_like(x)
        loss = plan.steps(x, m, v, 1, lr4, 400)
        fits.append((x.cpu().numpy().astype(np.float64), plan.loss_grad(x)[0].cpu().numpy()))
    (xt, lt), (xf, lf) = fits
    at, af = dp.unpack(xt)[2], dp.unpack(xf)[2]
    rel = np.abs(af - at) / np.abs(at)
    _say(f"pipeline deconv: chi2/2 true kernels {lt[0]:.4e}, fitted kernels {lf[0]:.4e}; "
         f"point amplitudes rel diff median {np.median(rel):.3e} max {rel.max():.3e}")
    # (measured: chi2 with the fitted kernels within 0.3 % of the true kernels' value,
    # amplitudes 2.9 % apart in the median, 6.7 % at most)
    assert lf[0] <= 1.05 * lt[0]
    assert np.median(rel) <= 0.05 and rel.max() <= 0.12


# --------------------------------------------------------------------------- #
# Shape classes on different algorithms in one plan; the autotuner             #
# --------------------------------------------------------------------------- #

# per class of the 10-epoch supernova subset (sides 32..128): direct, FFT one-launch
# forward, FFT line passes, in a rotation that gives every pattern a class
MIXES = {
    "dir-fused-lines": [(1, True), (2, True), (2, False)],
    "lines-dir-fused": [(2, False), (1, True), (2, True)],
}


def _mixed_plan(prob, d, w, mix):
    st = _st()
    plan = st.Plan.for_problem(prob, conv_algo=st.CONV_FFT)
    plan.set_frames(d, w, prob.kernels, prob.W)
    cls = plan.classes()
    for c in range(len(cls)):
        algo, fused = mix[c % len(mix)]
        plan.set_class_algo(c, algo, fused)
    got = plan.classes()
    assert {c["algo"] for c in got} == {1, 2}, got
    return plan, got


@pytest.mark.parametrize("mix", sorted(MIXES), ids=sorted(MIXES))
def test_mixed_class_algorithms_loss_grad_and_operators(mix):
    """Frames of some shape classes on the direct algorithm and the rest on the FFT
    algorithm (one-launch forward or line passes) in one evaluation: loss, gradient,
    the operators and their adjoint against the oracle."""
    prob = synth.make_deconv(4, E=10)
    d, w, rng = _data(prob, seed=41)
    plan, cls = _mixed_plan(prob, d, w, MIXES[mix])
    _say(f"mixed {mix}: " + ", ".join(f"n{c['n']}/K{c['K']}:{'dir' if c['algo'] == 1 else ('fused' if c['fused'] else 'lines')}"
                                        for c in cls))
    for point in ("init", "near"):
        p = synth.eval_point(prob, point, rng)
        _compare_loss_grad(prob, d, w, p, plan, f"mixed {mix}/{point}")
    scene = synth.f32(rng.standard_normal(prob.fine_size) * 30)
    model = plan.convolve_subsample(scene).cpu().numpy().astype(np.float64)
    ref = ora.conv_sub(prob.n, prob.K, prob.s, prob.kernels, scene)
    _check_frames(model, ref, prob.n.tolist(), 1e-5)
    resid = synth.f32(rng.standard_normal(prob.data_size))
    adj = plan.convolve_subsample_adj(resid).cpu().numpy().astype(np.float64)
    refa = ora.conv_sub_adj(prob.n, prob.K, prob.s, prob.kernels, resid)
    _check_frames(adj, refa, (prob.s * prob.n).tolist(), 1e-5)


def test_partial_adjoint_chunk_with_unwritten_spectra_slots():
    """A chunk of the frequency-domain adjoint with fewer frames than slots, in a plan
    whose first frames run the direct algorithm (their spectrum slots are never
    written): device memory is filled with NaN and released first, so that the plan's
    buffers start with non-finite values; the gradient must stay finite and match the
    oracle (regression: the missing slots once read frame 0's unwritten spectra and
    scaled them by zero)."""
    poison = torch.full((256 * 1024 * 1024,), float("nan"), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    del poison
    torch.cuda.empty_cache()
    prob = synth.make_deconv(4, E=10)
    d, w, rng = _data(prob, seed=42)
    plan, cls = _mixed_plan(prob, d, w, MIXES["dir-fused-lines"])
    assert cls[0]["algo"] == 1  # the first class (holding frame 0) on the direct algorithm
    p = synth.eval_point(prob, "near", rng)
    _, g = _compare_loss_grad(prob, d, w, p, plan, "partial chunk, poisoned memory")
    assert np.isfinite(g).all()


def test_mixed_class_algorithms_graph_steps_match_eager():
    """Optimiser steps of a mixed plan (the update fused into the final launch):
    graph replays equal eager steps bit for bit, and equal the all-FFT plan's loss
    up to rounding."""
    st = _st()
    prob = synth.make_deconv(4, E=10)
    d, w, rng = _data(prob, seed=42)
    p = torch.tensor(synth.eval_point(prob, "near", rng), dtype=torch.float32, device="cuda")
    plan_g, _ = _mixed_plan(prob, d, w, MIXES["dir-fused-lines"])
    plan_e, _ = _mixed_plan(prob, d, w, MIXES["dir-fused-lines"])
    plan_g.set_graph_mode(True)
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    xg, xe = p.clone(), p.clone()
    mg, vg, me, ve = (torch.zeros_like(p) for _ in range(4))
    lg = torch.empty(3, dtype=torch.float64, device="cuda")
    for t in range(1, 5):
        plan_g.step(xg, mg, vg, t, lr4, loss_out=lg)
        le = plan_e.step(xe, me, ve, t, lr4)
        torch.cuda.synchronize()
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()
        same = [torch.equal(a, b) for a, b in ((lg, le), (xg, xe), (mg, me), (vg, ve))]
        if not all(same):
            dx = (xg - xe).abs()
            _say(f"mixed graph step {t}: equal (loss, x, m, v) {same}; loss {lg.tolist()} vs {le.tolist()}; "
                 f"x differs at {int((dx > 0).sum())} entries, first {int(torch.nonzero(dx)[0])} of {dx.numel()}, "
                 f"max {dx.max().item():.3e}")
        assert all(same), t
    fft = st.Plan.for_problem(prob, conv_algo=st.CONV_FFT)
    fft.set_frames(d, w, prob.kernels, prob.W)
    lf, _ = fft.loss_grad(xe)
    lm, _ = plan_e.loss_grad(xe)
    assert abs(lf[2].item() - lm[2].item()) <= 1e-6 * abs(lf[2].item())


@pytest.mark.parametrize("case,fcs", [("cfg4_sub", (2, 4, 8)), ("cfg2_E5", (2, 4)), ("eleven_sources", (1, 2, 4)),
                                      ("seventeen_sources", (1, 2))])
def test_fft_adjoint_chunk_sizes(case, fcs):
    """The frequency-domain adjoint with 2, 4 and 8 frames per chunk (8 only with one
    point source), including a last chunk that is not full, against the oracle and
    against each other. Eleven sources: 1-frame chunks take sixteen sources per pass (one
    pass, not full), 2-frame chunks eight (a full pass and a pass of three), 4-frame chunks
    four (two full passes and one of three); seventeen: a full 16-source pass and one of one."""
    st = _st()
    if case == "cfg4_sub":
        prob = synth.make_deconv(4, E=13)
    elif case == "cfg2_E5":
        prob = synth.make_deconv(2, E=5)
    elif case == "eleven_sources":
        prob = synth.make_small_deconv(331, 5, [24, 32], [15, 21], 2, 80, 11, 4)
    else:
        prob = synth.make_small_deconv(332, 3, [20, 28], [13, 17], 3, 96, 17, 4)
    d, w, rng = _data(prob, seed=71)
    plan = _plan(prob, d, w, algo=st.CONV_FFT)
    p = synth.eval_point(prob, "near", rng)
    grads = []
    for fc in fcs:
        plan.set_fft_shapes(adj_frames=fc)
        assert plan.autotune_info()["adj_frames"] == fc
        _, g = _compare_loss_grad(prob, d, w, p, plan, f"{case}/adj_frames {fc}")
        grads.append(g)
    for g in grads[1:]:
        assert parity.rel_err(g, grads[0]) <= 1e-5
    for bad in (3, 16) + ((8,) if prob.M > 1 else ()) + ((1,) if prob.M <= 8 else ()):
        with pytest.raises(RuntimeError):
            plan.set_fft_shapes(adj_frames=bad)


def test_inplace_one_launch_forward():
    """Frames whose two LDS planes do not fit (128^2 data, Q = 160) take the one-launch
    forward with a single plane transformed in place: against the oracle, and against
    the same class on the line passes."""
    st = _st()
    prob = synth.make_deconv(4, E=13)
    d, w, rng = _data(prob, seed=73)
    plan = _plan(prob, d, w, algo=st.CONV_FFT)
    cls = plan.classes()
    big = [c for c, ci in enumerate(cls) if ci["n"] == 128]
    assert big and all(cls[c]["fused"] == 2 for c in big), cls
    assert all(ci["fused"] == 1 for ci in cls if ci["n"] < 128), cls
    p = synth.eval_point(prob, "near", rng)
    _, g_ip = _compare_loss_grad(prob, d, w, p, plan, "in-place forward")
    for c in big:
        plan.set_class_algo(c, st.CONV_FFT, fused=False)
    assert all(plan.classes()[c]["fused"] == 0 for c in big)
    _, g_lines = _compare_loss_grad(prob, d, w, p, plan, "line passes")
    assert parity.rel_err(g_ip, g_lines) <= 1e-5


@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_split_forward_is_bitwise_the_same(graph):
    """The one-launch forward on the plan's second FFT stream, beside the line passes,
    and the prior forked after the forward instead of at the start give bitwise the
    results of the in-order launches (loss, gradient and Adam steps, eager or captured),
    and match the oracle."""
    st = _st()
    prob = synth.make_deconv(4, E=13)
    d, w, rng = _data(prob, seed=72)
    plan = _plan(prob, d, w, algo=st.CONV_FFT)
    for c, ci in enumerate(plan.classes()):
        if ci["n"] == 128:  # the largest stamps onto the line passes
            plan.set_class_algo(c, st.CONV_FFT, fused=False)
    cls = plan.classes()
    assert any(c["fused"] for c in cls) and any(not c["fused"] for c in cls), cls
    p0 = synth.eval_point(prob, "near", rng)
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    runs = []
    for split, late in ((0, 0), (1, 0), (0, 1), (1, 1)):
        plan.set_fft_shapes(split_forward=split, prior_late=late)
        info = plan.autotune_info()
        assert info["split_forward"] == split and info["prior_late"] == late
        plan.set_graph_mode(graph)
        x = torch.tensor(p0, dtype=torch.float32, device="cuda")
        m = torch.zeros_like(x)
        v = torch.zeros_like(x)
        l, g = plan.loss_grad(x)
        l, g = l.clone(), g.clone()
        for t in range(1, 4):
            plan.step(x, m, v, t, lr4)
        torch.cuda.synchronize()
        runs.append((l, g, x.clone(), m.clone(), v.clone()))
        plan.set_graph_mode(False)
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert torch.equal(a, b)
    _compare_loss_grad(prob, d, w, p0, plan, "split forward, late prior")


@pytest.mark.parametrize("split", [0, 1])
def test_prior_riding_in_multi_class_launches(split):
    """Several FFT classes with the prior's passes carried by the evaluation's own launches
    (prior_late 2; the final launch sums the per-level terms per pixel): against the oracle,
    against the forked prior (rounding of the per-pixel sum only), and graph steps equal to
    eager ones; with the one-launch forward beside the line passes or in order."""
    st = _st()
    prob = synth.make_deconv(4, E=13)
    d, w, rng = _data(prob, seed=74)
    plan = _plan(prob, d, w, algo=st.CONV_FFT)
    if split:
        for c, ci in enumerate(plan.classes()):
            if ci["n"] == 128:
                plan.set_class_algo(c, st.CONV_FFT, fused=False)
    assert len(plan.classes()) > 1
    p0 = synth.eval_point(prob, "near", rng)
    plan.set_fft_shapes(split_forward=split, prior_late=1)
    lf, gf = plan.loss_grad(p0)
    lf, gf = lf.cpu().numpy(), gf.cpu().numpy().astype(np.float64)
    plan.set_fft_shapes(prior_late=2)
    assert plan.autotune_info()["prior_late"] == 2
    lr_, gr_ = plan.loss_grad(p0)
    lr_, gr_ = lr_.cpu().numpy(), gr_.cpu().numpy().astype(np.float64)
    assert abs(lr_[2] - lf[2]) <= 1e-12 * abs(lf[2])
    assert parity.rel_err(gr_, gf) <= 1e-6
    _compare_loss_grad(prob, d, w, p0, plan, f"riding prior, split {split}")
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    outs = []
    for graph in (False, True):
        plan.set_graph_mode(graph)
        x = torch.tensor(p0, dtype=torch.float32, device="cuda")
        m = torch.zeros_like(x)
        v = torch.zeros_like(x)
        for t in range(1, 4):
            plan.step(x, m, v, t, lr4)
        torch.cuda.synchronize()
        outs.append((x.clone(), m.clone(), v.clone()))
    plan.set_graph_mode(False)
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    # the fork after the adjoint's spectral products: bitwise the forked prior's results
    plan.set_fft_shapes(prior_late=3)
    l3, g3 = plan.loss_grad(p0)
    assert np.array_equal(l3.cpu().numpy(), lf) and np.array_equal(g3.cpu().numpy().astype(np.float64), gf)
    for bad in (4, -2):
        with pytest.raises(RuntimeError):
            plan.set_fft_shapes(prior_late=bad)


def test_autotuner_per_class_choices_cache_and_parity():
    """The automatic choice times each class's alternatives; a second plan of the same
    shapes takes the cached decision; the tuned plan matches the oracle."""
    st = _st()
    prob = synth.make_deconv(4, E=10)
    d, w, rng = _data(prob, seed=43)
    plan = st.Plan.for_problem(prob)
    plan.set_frames(d, w, prob.kernels, prob.W)
    info = plan.autotune_info()
    cls = plan.classes()
    _say(f"autotune: {info}; " + "; ".join(f"n{c['n']}: algo {c['algo']} fused {c['fused']} ms {c['tune_ms']}"
                                           for c in cls))
    assert info["wall_ms"] > 0
    for c in cls:
        tried = [v for v in c["tune_ms"] if v >= 0]
        assert len(tried) >= 2, c  # the current choice and at least one alternative
    plan2 = st.Plan.for_problem(prob)
    plan2.set_frames(d, w, prob.kernels, prob.W)
    info2 = plan2.autotune_info()
    assert info2["cached"] and [c["algo"] for c in plan2.classes()] == [c["algo"] for c in cls]
    assert info2["adj_blocks"] == info["adj_blocks"] and info2["line_groups"] == info["line_groups"]
    assert info2["adj_frames"] == info["adj_frames"]
    p = synth.eval_point(prob, "near", rng)
    _compare_loss_grad(prob, d, w, p, plan, "autotuned cfg4 subset")


# --------------------------------------------------------------------------- #
# Per-frame shifts and rotations                                               #
# --------------------------------------------------------------------------- #

XF_CASES = {
    # small ragged frames, two sources, odd and even kernels
    "small": lambda: synth.make_small_deconv(61, 4, [16, 24, 8, 20], [15, 16, 5, 9], 2, 64, 2, 4),
    # supernova stamps
    "cfg4_sizes": lambda: synth.make_deconv(4, E=6),
}


def _xf_for(E, rng, big=False):
    d = rng.uniform(-2.5, 2.5, (E, 2))
    th = rng.uniform(-0.6, 0.6, E) if not big else rng.uniform(-np.pi, np.pi, E)
    return synth.f32(np.column_stack([d, th]).ravel())


@pytest.mark.parametrize("xalgo", [1, 2], ids=["direct", "fft"])
@pytest.mark.parametrize("name", sorted(XF_CASES), ids=sorted(XF_CASES))
def test_frame_transforms_parity(name, xalgo):
    """Frames shifted and rotated, convolved by the direct kernels or through each
    frame's own spectrum: scenes element by element, loss, every gradient block and
    dL/d(dx, dy, theta) per frame against the oracle; clearing the transforms gives
    back the untransformed plan's results."""
    st = _st()
    prob = XF_CASES[name]()
    d, w, rng = _data(prob, seed=62)
    plan = _plan(prob, d, w, algo=st.CONV_AUTO)
    p = synth.eval_point(prob, "near", rng)
    l_plain, g_plain = plan.loss_grad(p)
    l_plain, g_plain = l_plain.clone(), g_plain.clone()
    for big in (False, True):
        xf = _xf_for(prob.E, rng, big)
        gx = plan.set_frame_transforms(xf, algo=xalgo)
        assert all(c["algo"] == st.CONV_DIRECT for c in plan.classes())
        assert plan.frame_transforms_info()[0] == xalgo
        sc = plan.render_scene(p).cpu().numpy().astype(np.float64)
        ref = ora.render_scene_xf(prob.n, prob.s, prob.N, prob.M, prob.fwhm, p, xf)
        _check_frames(sc, ref, (prob.s * prob.n).tolist(), 2e-6)
        loss, grad = plan.loss_grad(p)
        torch.cuda.synchronize()
        loss = loss.cpu().numpy()
        grad = grad.cpu().numpy().astype(np.float64)
        gxd = gx.cpu().numpy().astype(np.float64)
        NN = prob.N ** 2
        so, nsub = parity.tie_override(prob.N, prob.J, p[:NN], plan.starlet_fwd(p[:NN]).cpu().numpy())
        lo, go, gxo = ora.loss_grad_xf(prob, d, w, p, xf, sgn_override=so)
        rl = abs(loss[2] - lo[2]) / abs(lo[2])
        blocks = {k: parity.rel_err(parity.deconv_blocks(prob, grad)[k], v)
                  for k, v in parity.deconv_blocks(prob, go).items() if np.linalg.norm(v) > 0}
        rx = parity.rel_err(gxd, gxo)
        rxs = [parity.rel_err(gxd[j::3], gxo[j::3]) for j in range(3)]
        _say(f"xf {name}/{'fft' if xalgo == 2 else 'direct'} big={big}: loss rel {rl:.2e}; grad {blocks}; "
             f"transforms {rx:.2e} {rxs}")
        assert rl <= 1e-6
        assert parity.rel_err(grad, go) <= 1e-4
        for k, v in blocks.items():
            assert v <= 1e-4, (k, v)
        for j in range(3):
            assert rxs[j] <= 1e-4, j
    plan.set_frame_transforms(None)
    l2, g2 = plan.loss_grad(p)
    assert abs(l2[2].item() - l_plain[2].item()) <= 1e-6 * abs(l_plain[2].item())
    assert parity.rel_err(g2.cpu().numpy(), g_plain.cpu().numpy()) <= 1e-5


def test_frame_transforms_auto_choice_and_graph_steps():
    """With STARRED_CONV_AUTO the plan times both convolutions of the transformed frames
    and keeps the faster; optimiser steps with transforms replayed from a captured
    graph equal eager steps bit for bit, on both convolutions."""
    st = _st()
    prob = synth.make_deconv(4, E=6)
    d, w, rng = _data(prob, seed=63)
    xf = _xf_for(prob.E, rng)
    p = torch.tensor(synth.eval_point(prob, "near", rng), dtype=torch.float32, device="cuda")
    lr4 = [prob.adam_lr[k] for k in ("h", "Gamma", "a", "c")]
    plan = _plan(prob, d, w, algo=st.CONV_AUTO)
    plan.set_frame_transforms(xf)
    algo, ms = plan.frame_transforms_info()
    _say(f"transforms auto: algo {algo}, ms {ms}")
    assert ms["direct"] > 0 and ms["fft"] > 0
    assert algo == (st.CONV_FFT if ms["fft"] < ms["direct"] else st.CONV_DIRECT)
    for xalgo in (st.CONV_DIRECT, st.CONV_FFT):
        runs = []
        for graph in (False, True):
            pl = _plan(prob, d, w, algo=st.CONV_AUTO)
            gx = pl.set_frame_transforms(xf, algo=xalgo)
            pl.set_graph_mode(graph)
            x = p.clone()
            m = torch.zeros_like(p)
            v = torch.zeros_like(p)
            for t in range(1, 4):
                loss = pl.step(x, m, v, t, lr4)
                torch.cuda.synchronize()
                _ = (torch.randn(1000, device="cuda") * 2).sum().item()
            runs.append((loss.clone(), x.clone(), m.clone(), v.clone(), gx.clone()))
        for a, b in zip(*runs):
            assert torch.equal(a, b), xalgo


# --------------------------------------------------------------------------- #
# L-BFGS-B with device evaluations against scipy's on the oracle               #
# --------------------------------------------------------------------------- #

def _lbfgsb_tracks(fun_oracle, plan, x0, lo, hi, iters, label):
    import scipy.optimize
    xs_s = []
    res = scipy.optimize.minimize(fun_oracle, x0, jac=True, method="L-BFGS-B", bounds=list(zip(lo, hi)),
                                  options=dict(maxiter=iters, maxcor=10),
                                  callback=lambda xk: xs_s.append(np.array(xk, dtype=np.float64)))
    x = torch.tensor(x0, dtype=torch.float32, device="cuda")
    opt = plan.lbfgs(m=10, lo=lo.astype(np.float32), hi=hi.astype(np.float32))
    xs_d, fs_d = [], []
    for _ in range(iters):
        f, _ = opt.run(x, 1)
        xs_d.append(x.cpu().numpy().astype(np.float64))
        fs_d.append(f)
    k = min(len(xs_s), len(xs_d))
    errs = [np.abs(xs_d[i] - xs_s[i]).max() / max(np.abs(xs_s[i]).max(), 1.0) for i in range(k)]
    _say(f"{label}: iterate differences vs scipy " + " ".join(f"{e:.1e}" for e in errs))
    _say(f"{label}: loss device {fs_d[-1]:.9e} scipy {res.fun:.9e} after {iters} iterations")
    return errs, fs_d[-1], res.fun


def test_lbfgsb_device_iterates_track_scipy_deconvolution():
    """cfg1 (4 epochs of 32^2, lambda = 0) with h >= 0 and a_ik >= 0: the device-driven
    L-BFGS-B follows scipy's L-BFGS-B on the FP64 oracle iterate by iterate. The two
    evaluate the loss in FP32 and FP64, so the trajectories separate slowly: the first
    five iterates within 1e-4 of the largest entry, the loss after 20 iterations
    within 1e-3."""
    st = _st()
    prob = synth.make_deconv(1)
    d, w, rng = _data(prob, seed=83)
    plan = st.Plan.for_problem(prob, lam=0.0)
    plan.set_frames(d, w, prob.kernels, prob.W)
    NN, E, M = prob.N ** 2, prob.E, prob.M
    lo = np.full(prob.n_params, -np.inf)
    hi = np.full(prob.n_params, np.inf)
    lo[:NN] = 0.0
    lo[NN + E:NN + E + E * M] = 0.0
    x0 = synth.f32(np.maximum(synth.eval_point(prob, "init", rng), lo))

    def fun(q):
        loss, g = ora.loss_grad(prob, d, w, q, lam=0.0)
        return loss[2], g
    errs, fd, fs = _lbfgsb_tracks(fun, plan, x0, lo, hi, 20, "lbfgsb cfg1")
    assert max(errs[:5]) <= 1e-4
    assert abs(fd - fs) <= 1e-3 * abs(fs)


def test_lbfgsb_device_iterates_track_scipy_psf():
    """PSF mode (4 star stamps of 16^2, s = 3) with positive widths, exponent and
    amplitudes: the same comparison."""
    st = _st()
    prob = synth.make_psf(3, S=4, n=16, s=3, J=4)
    rng = np.random.default_rng(84)
    m = ora.psf_model(prob, prob.params_true)
    d, w = synth.add_noise(m, rng, poisson=False)
    plan = st.Plan.for_psf(prob)
    plan.set_frames(d, w, None, prob.W)
    NN, S = prob.N ** 2, prob.S
    lo = np.full(prob.n_params, -np.inf)
    hi = np.full(prob.n_params, np.inf)
    lo[1:3] = 0.5
    lo[4] = 1.0
    lo[5 + NN:5 + NN + S] = 0.0
    x0 = synth.f32(np.maximum(synth.psf_eval_point(prob, "init", rng), lo))

    def fun(q):
        loss, g = ora.psf_loss_grad(prob, d, w, q)
        return loss[2], g
    errs, fd, fs = _lbfgsb_tracks(fun, plan, x0, lo, hi, 20, "lbfgsb psf")
    assert max(errs[:5]) <= 1e-4
    assert abs(fd - fs) <= 1e-3 * abs(fs)


# --------------------------------------------------------------------------- #
# Edge cases: no point sources, a single starlet plane, sources at frame edges #
# --------------------------------------------------------------------------- #

def _edge_case(name):
    if name == "no_sources":
        return synth.make_small_deconv(91, 3, [16, 12, 20], [9, 8, 5], 2, 48, 0, 4)
    if name == "one_plane":
        prob = synth.make_small_deconv(92, 3, [16, 12, 20], [9, 8, 5], 2, 48, 1, 1)
        return synth.DeconvProblem(**{**prob.__dict__, "W": synth.f32([2.5])})
    # sources within 8 px of the windows' edges (and one just outside the smallest
    # window), where the +-8 px evaluation box of r meets the window crop
    prob = synth.make_small_deconv(93, 3, [16, 12, 20], [9, 8, 5], 2, 48, 3, 4)
    return synth.DeconvProblem(**{**prob.__dict__, "c": synth.f32([6.3, 20.7, 44.6, 30.2, 10.8, 13.1])})


@pytest.mark.parametrize("algo", ALGOS, ids=lambda a: ALGO_ID[a])
@pytest.mark.parametrize("name", ["no_sources", "one_plane", "sources_at_edges"])
def test_loss_grad_parity_edge_cases(name, algo):
    prob = _edge_case(name)
    d, w, rng = _data(prob, seed=94)
    plan = _plan(prob, d, w, algo)
    for point in ("init", "near"):
        p = synth.eval_point(prob, point, rng)
        _compare_loss_grad(prob, d, w, p, plan, f"edge {name}/{ALGO_ID[algo]}/{point}")
