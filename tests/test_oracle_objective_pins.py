"""Pins for the oracle of the packet-conditioned objective (Sec. 4, Eq. (2)):
each part against a closed form, a brute-force definition or an independent
implementation, and the image gradient against central differences."""

import numpy as np
import pytest
import torch

from oracle import objective as O
from oracle import utility as U


def _imgs(rng, K, H=9, W=11):
    return rng.uniform(0.0, 1.0, (K, H, W, 3))


def test_locked_constants_are_the_papers():
    # D = MSE + 0.20 (1 - SSIM); lambda_c 0.30 at CVaR_0.05; lambda_t 0.10; lambda_m 2.0; anchor 0.50
    assert O.LOCKED == dict(lambda_ssim=0.20, lambda_c=0.30, alpha=0.05, lambda_t=0.10, lambda_m=2.0, lambda_a=0.50)


def test_conv2d_ssim_equals_the_explicit_window_sums():
    """Two implementations: 121 explicit shifted sums (numpy) and conv2d (torch)."""
    rng = np.random.default_rng(3)
    for H, W in ((9, 11), (16, 5), (23, 31)):
        x = rng.uniform(0, 1, (H, W, 3))
        y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
        y[: H // 2] = 0.4  # flat region: zero variance windows
        a = float(O.ssim_t(torch.tensor(x), torch.tensor(y)))
        assert a == pytest.approx(U.ssim(x, y), abs=1e-13)
        d = float(O.distortion_t(torch.tensor(x), torch.tensor(y)))
        assert d == pytest.approx(U.distortion(x, y), abs=1e-13)
    assert float(O.ssim_t(torch.tensor(x), torch.tensor(x))) == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("n,alpha", [(5, 0.4), (5, 0.3), (40, 0.05), (30, 0.05), (7, 0.1), (8, 1.0), (3, 0.999)])
def test_cvar_matches_rockafellar_uryasev_minimum(n, alpha):
    """CVaR_alpha = min_tau tau + (1/(alpha n)) sum (D - tau)_+ ; the function
    is convex and piecewise linear in tau with kinks at the data, so its
    minimum sits at one of the data values."""
    rng = np.random.default_rng(n)
    d = rng.uniform(0, 1, n)
    ru = min(t + np.maximum(d - t, 0.0).sum() / (alpha * n) for t in d)
    got = float(O.cvar_upper(torch.tensor(d), alpha))
    assert got == pytest.approx(ru, abs=1e-12)


def test_cvar_closed_forms_and_special_cases():
    d = torch.tensor([0.1, 0.5, 0.3, 0.9, 0.2], dtype=torch.float64)
    assert float(O.cvar_upper(d, 0.4)) == pytest.approx((0.9 + 0.5) / 2)          # alpha n = 2
    assert float(O.cvar_upper(d, 0.3)) == pytest.approx((0.9 + 0.5 * 0.5) / 1.5)  # alpha n = 1.5
    assert float(O.cvar_upper(d, 0.05)) == pytest.approx(0.9)                     # alpha n < 1: the maximum
    assert float(O.cvar_upper(d, 1.0)) == pytest.approx(float(d.mean()))          # the whole set: the mean
    same = torch.full((20,), 0.37, dtype=torch.float64)
    assert float(O.cvar_upper(same, 0.05)) == pytest.approx(0.37)


def test_monotonicity_hinge_and_temporal_closed_forms():
    H, W = 6, 7
    tg = np.stack([np.full((H, W, 3), 0.1), np.full((H, W, 3), 0.3)])
    imgs = np.stack([np.full((H, W, 3), 0.2), np.full((H, W, 3), 0.5)])
    # temporal: (I_1 - I_0) - (G_1 - G_0) = 0.3 - 0.2 = 0.1 everywhere -> F = 0.01
    r = O.objective(imgs, tg, [0, 1], [], temporal=[(0, 1)], weights=dict(lambda_t=1.0), grad=False)
    assert r["F"] == pytest.approx(0.01, abs=1e-14) and r["loss"] == pytest.approx(0.01, abs=1e-14)
    # monotonicity: image 0 equals its target (D = 0); M averages the three hinges
    rng = np.random.default_rng(2)
    x = _imgs(rng, 3)
    t = x[0:1].copy()
    r = O.objective(x, t, [0, 0, 0], [], mono=[(0, 1), (1, 2), (2, 1)], grad=False)
    D = r["D"]
    assert D[0] == pytest.approx(0.0, abs=1e-14)
    want = (max(0.0, D[1] - D[0]) + max(0.0, D[2] - D[1]) + max(0.0, D[1] - D[2])) / 3
    assert r["M"] == pytest.approx(want, abs=1e-14) and r["M"] > 0


def test_parts_combine_with_the_weights():
    rng = np.random.default_rng(5)
    K = 9
    x = _imgs(rng, K)
    t = _imgs(rng, 2)
    tof = [0] * 5 + [1] * 4
    expect, anchor = [0, 1, 2, 3, 5, 6, 7], [4, 8]
    mono = [(0, 4), (1, 4), (5, 8)]
    temporal = [(0, 5), (1, 6), (4, 8)]
    r = O.objective(x, t, tof, expect, anchor, mono, temporal, grad=False)
    D = r["D"]
    for k in range(K):
        assert D[k] == pytest.approx(U.distortion(x[k], t[tof[k]]), abs=1e-13)
    De = D[expect]
    assert r["E"] == pytest.approx(De.mean(), abs=1e-14)
    srt = np.sort(De)[::-1]
    a = 0.05 * len(De)  # < 1: the worst value
    assert r["cvar"] == pytest.approx(srt[0], abs=1e-14) and a < 1
    assert r["anchor"] == pytest.approx(D[anchor].mean(), abs=1e-14)
    L = r["E"] + 0.3 * r["cvar"] + 0.1 * r["F"] + 2.0 * r["M"] + 0.5 * r["anchor"]
    assert r["loss"] == pytest.approx(L, abs=1e-14)


def test_image_gradient_matches_central_differences():
    rng = np.random.default_rng(9)
    K, H, W = 5, 7, 6
    x = _imgs(rng, K, H, W)
    t = _imgs(rng, 2, H, W)
    tof = [0, 0, 0, 1, 1]
    args = dict(expect=[0, 1, 3], anchor=[2], mono=[(0, 2), (3, 4)], temporal=[(0, 3), (2, 4)])
    wts = dict(alpha=0.5)  # alpha n = 1.5: one full and one half weight in the tail
    r = O.objective(x, t, tof, weights=wts, **args)
    g = r["grad"]
    h = 1e-6
    idx = [(k, int(rng.integers(H)), int(rng.integers(W)), int(rng.integers(3))) for k in range(K) for _ in range(6)]
    for (k, i, j, c) in idx:
        xp, xm = x.copy(), x.copy()
        xp[k, i, j, c] += h
        xm[k, i, j, c] -= h
        fd = (O.objective(xp, t, tof, weights=wts, grad=False, **args)["loss"] -
              O.objective(xm, t, tof, weights=wts, grad=False, **args)["loss"]) / (2 * h)
        assert g[k, i, j, c] == pytest.approx(fd, abs=1e-8, rel=1e-5), (k, i, j, c)
    # images in no role get no gradient
    r2 = O.objective(x, t, tof, [0], grad=True)
    assert np.all(r2["grad"][1:] == 0.0) and np.abs(r2["grad"][0]).max() > 0
