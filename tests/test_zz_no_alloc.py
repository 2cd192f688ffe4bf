"""The entry point that allocates nothing (starred_starlet_fwd_noalloc): its
coefficients against starred_starlet_fwd's on two calls in a row, the second
smaller, and the size limit of its fixed working array."""
import ctypes

import numpy as np
import pytest

from paper_2402_08725_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _plan_transform(N, J, img):
    from paper_2402_08725_amd import starred as st
    n = 10 if N % 2 == 0 else 9  # one frame whose window fits the grid with an integer offset
    plan = st.Plan(st.DECONV, [n], [3], 2 if N % 2 == 0 else 1, N, 0, J, 3.0)
    out = plan.starlet_fwd(img)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("first,second", [((300, 6), (64, 4)), ((512, 9), (33, 1))])
def test_noalloc_starlet_matches_the_plan_call(first, second):
    from paper_2402_08725_amd import starred as st
    rng = np.random.default_rng(71)
    for N, J in (first, second):
        print(f"noalloc starlet N={N} J={J}", flush=True)
        img = torch.tensor(synth.f32(rng.normal(0, 10, N * N) + 50.0), dtype=torch.float32, device="cuda")
        out = torch.full((J * N * N,), -7.0, dtype=torch.float32, device="cuda")
        st.starlet_fwd_noalloc(N, J, img, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        ref = _plan_transform(N, J, img)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"  max rel err vs plan {err:.2e}", flush=True)
        assert err <= 1e-6
        # exact reconstruction: the planes sum to the image
        rec = got.reshape(J, N, N).sum(axis=0).ravel()
        imgh = img.cpu().numpy().astype(np.float64)
        assert np.abs(rec - imgh).max() <= 1e-4 * np.abs(imgh).max()


def test_noalloc_starlet_rejects_sizes_beyond_its_array():
    from paper_2402_08725_amd import starred as st
    img = torch.zeros(520 * 520, dtype=torch.float32, device="cuda")
    out = torch.zeros(3 * 520 * 520, dtype=torch.float32, device="cuda")
    with pytest.raises(st.StarredError) as e:
        st.starlet_fwd_noalloc(520, 3, img, out)
    assert e.value.code == st.EINVAL
    with pytest.raises(st.StarredError):
        st.starlet_fwd_noalloc(64, 8, img, out)  # 2^(J-1) > N-1
