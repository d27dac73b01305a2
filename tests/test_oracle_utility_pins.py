"""Pins of the counterfactual-utility oracle (Eq. (3)-(4), D of Sec. 4)
against closed forms, a library filter and hand-computed values."""

import numpy as np
import pytest
import scipy.ndimage

import oracle
from oracle import utility as U
from scenes_for_tests import centred_camera, logit, scene_from_lists

BG = np.array([0.25, 0.5, 0.75])


def test_window_is_the_normalised_gaussian():
    w = U.ssim_window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w.T) and w[5, 5] == w.max()
    # separable: outer product of the 1D normalised Gaussian
    r = np.arange(-5, 6)
    g = np.exp(-r * r / 4.5)
    g /= g.sum()
    assert np.allclose(w, np.outer(g, g), rtol=0, atol=1e-16)


def test_ssim_identity_symmetry_and_constant_closed_form():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (20, 23, 3))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    assert abs(U.ssim(x, x) - 1.0) < 1e-12
    assert abs(U.ssim(x, y) - U.ssim(y, x)) < 1e-15
    assert U.ssim(x, y) < 1.0
    # constant images: away from the zero padding, sigma = 0 and
    # SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    m = U.ssim_map(np.full((16, 16, 3), a), np.full((16, 16, 3), b))
    want = (2 * a * b + U.SSIM_C1) / (a * a + b * b + U.SSIM_C1)
    assert np.abs(m[5:-5, 5:-5] - want).max() < 1e-12


def test_ssim_equals_the_library_gaussian_filter_with_zero_padding():
    """The window means are a truncated (radius 5) Gaussian filter with zero
    padding: scipy.ndimage.gaussian_filter(mode='constant') computes the same."""
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (19, 27, 3))
    y = rng.uniform(0, 1, (19, 27, 3))

    def f(z):
        return scipy.ndimage.gaussian_filter(z, sigma=(1.5, 1.5, 0), truncate=10.0 / 3.0, mode="constant", cval=0.0)

    mx, my = f(x), f(y)
    sxx, syy, sxy = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    lib = ((2 * mx * my + U.SSIM_C1) * (2 * sxy + U.SSIM_C2)) / ((mx ** 2 + my ** 2 + U.SSIM_C1) * (sxx + syy + U.SSIM_C2))
    assert np.abs(U.ssim_map(x, y) - lib).max() < 1e-12


def test_distortion_definition():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (12, 12, 3))
    y = rng.uniform(0, 1, (12, 12, 3))
    assert U.distortion(x, x) == pytest.approx(0.0, abs=1e-14)
    d = U.distortion(x, y)
    assert d == pytest.approx(np.mean((x - y) ** 2) + 0.2 * (1 - U.ssim(x, y)), rel=1e-14)
    assert U.distortion(x, y, lam=0.0) == pytest.approx(np.mean((x - y) ** 2), rel=1e-14)


def test_quantile_and_risk_adjusted_hand_values():
    v = np.arange(1, 11, dtype=np.float64)            # 1..10
    assert U.quantile_linear(v, 0.1) == pytest.approx(1.9, abs=1e-15)   # h = 0.9
    assert U.quantile_linear(v[::-1], 0.1) == pytest.approx(1.9, abs=1e-15)
    assert U.quantile_linear([4.0], 0.1) == 4.0
    rng = np.random.default_rng(4)
    for n in (2, 7, 31, 100):
        r = rng.normal(size=n)
        assert U.quantile_linear(r, 0.1) == pytest.approx(np.quantile(r, 0.1, method="linear"), abs=1e-14)
    s = U.risk_adjusted(v)
    std = np.sqrt(8.25)                                 # population variance of 1..10
    assert s["mean"] == 5.5 and s["std"] == pytest.approx(std, rel=1e-15)
    assert s["risk_adjusted"] == pytest.approx((0.75 * 5.5 + 0.25 * 1.9) / (1 + 0.05 * std), rel=1e-14)
    c = U.risk_adjusted(np.full(9, -0.3))
    assert c["risk_adjusted"] == pytest.approx(-0.3, abs=1e-15) and c["std"] == 0.0


def _group_scene():
    """Two packets: packet 0 = 3 Gaussians near the axis; packet 1 = one
    Gaussian off to the side (layer 0) and one behind the camera (layer 1)."""
    means = [[0.0, 0.0, 0.0], [0.05, -0.04, 0.2], [-0.06, 0.03, -0.1], [0.3, 0.25, 0.0], [0.0, 0.0, -5.0]]
    pl = [0 << 2 | 0, 0 << 2 | 1, 0 << 2 | 2, 1 << 2 | 0, 1 << 2 | 1]
    cols = [[0.9, 0.1, 0.1], [0.1, 0.8, 0.2], [0.2, 0.3, 0.9], [0.7, 0.7, 0.1], [1.0, 1.0, 1.0]]
    return scene_from_lists(means, -2.3, logits=[logit(0.8)] * 5, colors=cols, packet_layer=pl,
                            clusters=1, contexts=2)


def test_delta_special_cases():
    sc = _group_scene()
    cam = centred_camera(24, 24)
    basis = (0.0, 0.0)
    # every context holds packet 0 at depth 1 and packet 1 at depth 1
    ctx = np.array([[1, 1], [1, 1]], np.uint8)
    full = oracle.render(sc, cam, basis, np.array([[4, 4]], np.uint8), BG)["image"][0]
    # g = (packet 1, layer 1): its only Gaussian is behind the camera -> Delta = 0 exactly
    d = U.deltas(sc, cam, basis, ctx, 1, 1, full, BG)
    assert np.all(d == 0.0)
    # g = (packet 0, layer 1) against the reference R(m u g): Delta = D(I, R(m)) > 0
    ref = oracle.render(sc, cam, basis, np.array([[2, 1]], np.uint8), BG)["image"][0]
    d = U.deltas(sc, cam, basis, ctx[:1], 0, 1, ref, BG)
    m_img = oracle.render(sc, cam, basis, ctx[:1], BG)["image"][0]
    assert d[0] == pytest.approx(U.distortion(m_img, ref), rel=1e-15) and d[0] > 0
    # a context that already holds the group (or lacks its prerequisite) is rejected
    with pytest.raises(ValueError):
        U.paired_states(np.array([[2, 1]], np.uint8), 0, 1)
    with pytest.raises(ValueError):
        U.paired_states(np.array([[0, 1]], np.uint8), 0, 1)


def test_delta_is_local_to_the_group():
    """Pixels the group's Gaussians do not reach are identical in R(m) and
    R(m u g), so Eq. (3) equals the same difference over any region holding
    every changed pixel and its SSIM window."""
    sc = _group_scene()
    cam = centred_camera(32, 32)
    ref = np.random.default_rng(5).uniform(0, 1, (32, 32, 3))
    m, mg = U.paired_states(np.array([[1, 0]], np.uint8), 1, 0)
    assert mg.tolist() == [[1, 1]]
    a = oracle.render(sc, cam, (0.0, 0.0), m, BG)["image"][0]
    b = oracle.render(sc, cam, (0.0, 0.0), mg, BG)["image"][0]
    changed = np.any(a != b, axis=-1)
    assert changed.any() and not changed.all()
    ys, xs = np.nonzero(changed)
    y0, y1, x0, x1 = max(ys.min() - 5, 0), ys.max() + 6, max(xs.min() - 5, 0), xs.max() + 6
    full = U.deltas(sc, cam, (0.0, 0.0), m, 1, 0, ref, BG)[0]
    sa, sb = U.ssim_map(a, ref), U.ssim_map(b, ref)
    local = (((a - ref) ** 2 - (b - ref) ** 2)[y0:y1, x0:x1].sum()
             - 0.2 * (sa - sb)[y0:y1, x0:x1].sum()) / a.size
    assert full == pytest.approx(local, rel=1e-9, abs=1e-15)
    outside = np.ones_like(changed)
    outside[y0:y1, x0:x1] = False
    assert np.all((sa == sb)[outside])


def test_refined_deltas_reduce_to_plain_with_zero_levels():
    """Refinement levels of zero leave every state's render, so every delta,
    unchanged; non-zero levels of the group's packet change the delta."""
    import synth
    sc = synth.make_scene(300, 2, 2, 4, "rgb", index=8, stream=0)
    cam = centred_camera(24, 20)
    basis = synth.temporal_basis(0.5, sc.rank)
    ref = np.random.default_rng(1).uniform(0, 1, (20, 24, 3))
    ctx = np.array([[2, 1, 4, 0], [2, 3, 1, 1], [2, 0, 0, 4]], np.uint8)
    plain = U.deltas(sc, cam, basis, ctx, 0, 2, ref, BG)
    zero = U.deltas(sc, cam, basis, ctx, 0, 2, ref, BG, refine=np.zeros((3, oracle.refine_rows(0), sc.n), np.float32))
    assert np.array_equal(plain, zero)
    lv = synth.make_refinement(sc, index=8)
    refined = U.deltas(sc, cam, basis, ctx, 0, 2, ref, BG, refine=lv)
    assert np.abs(refined - plain).max() > 1e-6
