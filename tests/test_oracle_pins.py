"""Pins for the oracle: closed forms, invariants, brute force and library
routines -- checks that do not re-run the oracle's own formulas.

Sections of the paper these follow: Sec. 3 (Eq. (1) deformation; base + three
refinement groups per cluster), Sec. 4 (cluster-layer masks after dependency
enforcement), Sec. 6 (masked states rendered from one scene; FP32
rasterisation).  Rendering conventions the paper leaves open (projection,
1/255 skip, 0.99 cap, stop after T < 1e-4, +0.3 px^2 dilation, pixel centres at
+0.5) are pinned here as stated readings.
"""

import math
from dataclasses import replace

import numpy as np
import pytest

import oracle
import synth
from tests.scenes_for_tests import centred_camera, logit, overlap_scene, scene_from_lists

BG = np.array([0.25, 0.5, 0.75], np.float32)
BG64 = BG.astype(np.float64)
BASIS0 = np.zeros(2, np.float32)


def _o(lg32):
    return 1.0 / (1.0 + math.exp(-float(np.float32(lg32))))


# ----------------------------------------------------------------- exp_f32

def test_exp_f32_within_two_ulp():
    xs = np.linspace(-20.0, 10.0, 4001).astype(np.float32)
    for x in xs:
        got = oracle.exp_f32(float(x))
        ref = math.exp(float(x))
        ulp = np.spacing(np.float32(ref))
        assert abs(float(got) - ref) <= 2 * ulp, (x, got, ref)
    assert oracle.exp_f32(0.0) == np.float32(1.0)


# ------------------------------------------------------- P1 closed forms

def test_single_isotropic_gaussian_on_axis_closed_form():
    s_log = math.log(0.2)
    rng = np.random.default_rng(1)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    o = 0.8
    col = [0.9, 0.2, 0.4]
    sc = scene_from_lists([[0, 0, 0]], [s_log] * 3, [q], [logit(o)], [col])
    cam = synth.ring_camera(64, 64)
    codes = np.ones((1, 1), np.uint8)
    r = oracle.render(sc, cam, BASIS0, codes, BG)
    f = float(cam.fx)
    s2 = math.exp(2.0 * float(sc.log_scale[0, 0]))
    sig2 = f * f * s2 / 9.0 + 0.3
    oo = _o(sc.opacity_logit[0])
    colf = sc.color[:, 0].astype(np.float64)
    exp_img = np.zeros((64, 64, 3))
    exp_T = np.ones((64, 64))
    for py in range(64):
        for px in range(64):
            r2 = (px + 0.5 - cam.cx) ** 2 + (py + 0.5 - cam.cy) ** 2
            a = min(0.99, oo * math.exp(-r2 / (2.0 * sig2)))
            if a >= 1.0 / 255.0:
                exp_img[py, px] = a * colf + (1 - a) * BG64
                exp_T[py, px] = 1 - a
            else:
                exp_img[py, px] = BG64
    np.testing.assert_allclose(r["image"][0], exp_img, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["tfinal"][0], exp_T, rtol=0, atol=1e-12)
    # pixel centres at +0.5: the four central pixels are equally bright
    c = r["image"][0]
    assert np.allclose(c[31, 31], c[32, 32]) and np.allclose(c[31, 32], c[32, 31])


def test_off_axis_isotropic_jacobian_closed_form():
    s = 0.1
    # theta = 0 camera: camera x = -world x, camera z = world z + 3
    sc = scene_from_lists([[-0.3, 0, 0], [-2.5, 0, 0]], [math.log(s)] * 3)
    cam = synth.ring_camera(64, 48)
    g = oracle.geometry_f64(sc, cam, BASIS0)
    f = float(cam.fx)
    s2 = math.exp(2.0 * float(sc.log_scale[0, 0]))
    X = 0.3 * 1.0
    X = float(np.float32(-0.3)) * -1.0
    Z = 3.0
    assert g["X"][0] == pytest.approx(X, abs=1e-15) and g["Z"][0] == pytest.approx(Z, abs=1e-15)
    a = s2 * f * f * (1 / Z ** 2 + X ** 2 / Z ** 4) + 0.3
    c = s2 * f * f / Z ** 2 + 0.3
    assert g["a"][0] == pytest.approx(a, rel=1e-12)
    assert g["c"][0] == pytest.approx(c, rel=1e-12)
    assert abs(g["b"][0]) < 1e-12
    assert g["u"][0] == pytest.approx(f * X / Z + cam.cx, rel=1e-13)
    # second Gaussian: X/Z = 0.833 beyond 1.3 x tan(30 deg) = 0.7506 -> the
    # Jacobian's third column uses the clamped ratio, u keeps the true one
    X2 = float(np.float32(-2.5)) * -1.0
    lim = 1.3 * 64 / (2 * f)
    a2 = s2 * f * f * (1 / Z ** 2 + lim ** 2 / Z ** 2) + 0.3
    assert g["a"][1] == pytest.approx(a2, rel=1e-12)
    assert g["u"][1] == pytest.approx(f * X2 / Z + cam.cx, rel=1e-13)
    m = oracle.mirror_f32(sc, cam, BASIS0)
    assert m["a"][0] == pytest.approx(a, rel=2e-6) and m["c"][0] == pytest.approx(c, rel=2e-6)


def test_diagonal_offset_gaussian_covariance_and_conic():
    """Camera-frame mean (X, Y, Z) with X, Y != 0: the 2D covariance gains
    the cross term s^2 fx fy X Y / Z^4 (the sign pins both Jacobian columns),
    and every pixel follows alpha = o exp(-d^T Sigma2D^-1 d / 2) with the
    inverse taken by numpy.linalg.inv."""
    s = 0.12
    sc = scene_from_lists([[-0.3, -0.2, 0.0]], [math.log(s)] * 3, None, [logit(0.7)], [[0.2, 0.9, 0.4]])
    cam = synth.ring_camera(64, 64)
    g = oracle.geometry_f64(sc, cam, BASIS0)
    f = float(cam.fx)
    s2 = math.exp(2.0 * float(sc.log_scale[0, 0]))
    X, Y, Z = -float(np.float32(-0.3)), -float(np.float32(-0.2)), 3.0
    S = np.array([[s2 * f * f * (1 / Z ** 2 + X * X / Z ** 4) + 0.3, s2 * f * f * X * Y / Z ** 4],
                  [s2 * f * f * X * Y / Z ** 4, s2 * f * f * (1 / Z ** 2 + Y * Y / Z ** 4) + 0.3]])
    assert [g["a"][0], g["b"][0], g["c"][0]] == pytest.approx([S[0, 0], S[0, 1], S[1, 1]], rel=1e-12)
    Q = np.linalg.inv(S)
    u, v = f * X / Z + cam.cx, f * Y / Z + cam.cy
    pix = np.array([[int(u) + dx, int(v) + dy] for dx in range(-6, 7, 2) for dy in range(-6, 7, 3)])
    r = oracle.render(sc, cam, BASIS0, np.ones((1, 1), np.uint8), BG, pixels=pix)
    oo = _o(sc.opacity_logit[0])
    for k, (px, py) in enumerate(pix):
        d = np.array([u - (px + 0.5), v - (py + 0.5)])
        a = min(0.99, oo * math.exp(-0.5 * d @ Q @ d))
        exp = a * sc.color[:, 0].astype(np.float64) + (1 - a) * BG64 if a >= 1 / 255 else BG64
        np.testing.assert_allclose(r["image"][0, k], exp, atol=1e-12)


# ------------------------------------------------- P3 order and stopping

def _axis_scene(zs, opac, cols):
    return scene_from_lists([[0, 0, z] for z in zs], [math.log(0.3)] * 3, None,
                            [logit(o) for o in opac], cols)


def test_two_gaussian_composite_and_order():
    cam = centred_camera(32, 32, cx=16.5, cy=16.5)  # pixel (16,16) centre on the axis
    cols = [[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]
    pix = np.array([[16, 16]])
    codes = np.ones((1, 1), np.uint8)
    for zs, first in (([-0.5, 0.5], 0), ([0.5, -0.5], 1), ([0.0, 0.0], 0)):
        sc = _axis_scene(zs, [0.6, 0.7], cols)
        r = oracle.render(sc, cam, BASIS0, codes, BG, pixels=pix)
        o = [_o(sc.opacity_logit[k]) for k in range(2)]
        c = [sc.color[:, k].astype(np.float64) for k in range(2)]
        a1, a2 = o[first], o[1 - first]
        c1, c2 = c[first], c[1 - first]
        exp = a1 * c1 + (1 - a1) * a2 * c2 + (1 - a1) * (1 - a2) * BG64
        np.testing.assert_allclose(r["image"][0, 0], exp, atol=1e-12)
        assert r["ncomp"][0, 0] == 2


def test_include_then_stop():
    cam = centred_camera(16, 16, cx=8.5, cy=8.5)
    cols = [[k / 6.0, 1 - k / 6.0, 0.5] for k in range(6)]
    sc = _axis_scene([-0.5 + 0.2 * k for k in range(6)], [0.95] * 6, cols)
    r = oracle.render(sc, cam, BASIS0, np.ones((1, 1), np.uint8), BG, pixels=np.array([[8, 8]]))
    T, C = 1.0, np.zeros(3)
    for k in range(4):  # T after 4 Gaussians: 0.05^4 = 6.25e-6 < 1e-4 -> stop
        a = _o(sc.opacity_logit[k])
        C += T * a * sc.color[:, k].astype(np.float64)
        T *= 1 - a
    C += T * BG64
    np.testing.assert_allclose(r["image"][0, 0], C, atol=1e-12)
    assert r["ncomp"][0, 0] == 4
    assert r["tfinal"][0, 0] == pytest.approx(T, rel=1e-12)


def test_alpha_cap_and_skip():
    cam = centred_camera(16, 16, cx=8.5, cy=8.5)
    sc = _axis_scene([0.0], [0.999], [[1, 1, 1]])
    r = oracle.render(sc, cam, BASIS0, np.ones((1, 1), np.uint8), BG, pixels=np.array([[8, 8]]))
    assert r["tfinal"][0, 0] == pytest.approx(0.01, rel=1e-12)  # alpha capped at 0.99
    sc = _axis_scene([0.0], [0.003], [[1, 1, 1]])  # o < 1/255 everywhere -> skipped
    r = oracle.render(sc, cam, BASIS0, np.ones((1, 1), np.uint8), BG)
    assert np.all(r["image"][0] == BG.astype(np.float64)) and np.all(r["ncomp"] == 0)


# ------------------------------------------------ ambiguity budget pins
# The budget marks (state, pixel) pairs where an FP32 renderer may take the
# other branch of the 1/255 skip or of the T < 1e-4 stop, and bounds the image
# change: 2 T alpha M for a skip, 2 T_after (1 + relT) M for a stop, M = the
# largest |colour| or |background| (+ 2^-16).  The skip window is the FP32
# exponent's error bound: for a Gaussian seen at its own centre (dx = dy = 0)
# it is 8 2^-24 |log2 o| + 2^-16 in log2 units, i.e. about 1.3e-5 relative in
# alpha -- so an alpha 2e-6 from 1/255 is ambiguous and one 1e-4 away is not.

def _at_centre(alphas, cols, zs=None):
    """Gaussians on the optical axis seen at pixel (8, 8), whose centre is the
    principal point: |dx|, |dy| are rounding-level, so alpha = o to ~1e-7."""
    cam = centred_camera(16, 16, cx=8.5, cy=8.5)
    zs = [-0.5 + 0.1 * k for k in range(len(alphas))] if zs is None else zs
    sc = _axis_scene(zs, alphas, cols)
    r = oracle.render(sc, cam, BASIS0, np.ones((1, 1), np.uint8), BG, pixels=np.array([[8, 8]]))
    return sc, r


def _m(cols):
    return max(max(abs(c) for col in cols for c in col), float(np.max(np.abs(BG64)))) + 2.0 ** -16


@pytest.mark.parametrize("rel,amb", [(2e-6, True), (-2e-6, True), (1e-4, False), (-1e-4, False),
                                     (5e-4, False)])
def test_budget_skip_window(rel, amb):
    cols = [[0.9, 0.1, 0.3]]
    sc, r = _at_centre([(1 + rel) / 255.0], cols)
    a = _o(sc.opacity_logit[0])
    assert abs(a * 255.0 - 1.0 - rel) < 5e-7  # FP32 logit moves alpha by < 4e-7
    B = r["budget"][0, 0]
    if amb:
        assert B == pytest.approx(2.0 * a * _m(cols), rel=1e-6)
    else:
        assert B == 0.0
    # the definition itself: composited iff alpha >= 1/255
    assert r["ncomp"][0, 0] == (1 if a >= 1 / 255 else 0)


def test_budget_stop_window():
    cols = [[0.2, 0.4, 0.6], [0.7, 0.1, 0.5], [0.3, 0.3, 0.9]]
    # two capped alphas leave T = (1 - 0.99)^2 = 1e-4 (+2e-18): either side of the stop
    sc, r = _at_centre([0.9999, 0.9999], cols[:2])
    Ta = (1 - 0.99) ** 2
    assert r["ncomp"][0, 0] == 2 and r["tfinal"][0, 0] == pytest.approx(Ta, rel=1e-12)
    assert r["budget"][0, 0] == pytest.approx(2.0 * Ta * _m(cols[:2]), rel=1e-3)
    # T far from 1e-4 after each composited Gaussian: no budget
    sc, r = _at_centre([0.9999, 0.95, 0.9], cols)
    assert r["ncomp"][0, 0] == 3 and r["budget"][0, 0] == 0.0
    sc, r = _at_centre([0.9999, 0.5], cols[:2])
    assert r["budget"][0, 0] == 0.0


def _third_alpha(t1, target):
    """alpha of a third Gaussian that takes T from t1 * 0.01 to target."""
    return 1.0 - target / (t1 * (1 - 0.99))


def test_budget_earlier_ambiguous_skip_widens_stop_window():
    """T after three Gaussians lands 0.25% above 1e-4.  Alone, that is outside
    the stop window (whose width is the alphas' FP32 error, ~1e-3 here); after
    a Gaussian whose skip may flip (changing T by up to alpha / (1 - alpha) =
    0.4%) it is inside, and the stop term appears."""
    cols = [[0.2, 0.4, 0.6], [0.7, 0.1, 0.5], [0.3, 0.3, 0.9]]
    target = 1e-4 * (1 + 2.5e-3)
    # ambiguous first alpha (2e-6 above 1/255)
    a1 = (1 + 2e-6) / 255.0
    sc, r = _at_centre([a1, 0.9999, _third_alpha(1 - a1, target)], cols)
    o1 = _o(sc.opacity_logit[0])
    T = (1 - o1) * (1 - 0.99) * (1 - _o(sc.opacity_logit[2]))
    assert T == pytest.approx(target, rel=1e-5) and r["ncomp"][0, 0] == 3
    skip_term = 2.0 * o1 * _m(cols)
    B = r["budget"][0, 0]
    assert 2.0 * T * _m(cols) < B - skip_term < 2.02 * T * _m(cols)
    # the same T after a first alpha that is clearly above 1/255: no budget at all
    a1 = 1.05 / 255.0
    sc, r = _at_centre([a1, 0.9999, _third_alpha(1 - a1, target)], cols)
    T = (1 - _o(sc.opacity_logit[0])) * (1 - 0.99) * (1 - _o(sc.opacity_logit[2]))
    assert T == pytest.approx(target, rel=1e-5) and r["budget"][0, 0] == 0.0


def test_budget_share_on_the_tiny_workload():
    """On the 4,096-Gaussian 128x128 16-state workload the budget excuses
    fewer than 0.1% of (state, pixel) pairs, none by more than 0.01."""
    w = synth.make_workload("g4k_128px_16states", background=BG)
    B = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background)["budget"]
    assert 0 < (B > 0).mean() < 1e-3
    assert B.max() < 1e-2


# ------------------------------------------------------ P4-P7 invariants

@pytest.fixture(scope="module")
def tiny():
    return synth.make_workload("g4k_128px_16states", background=BG)


def test_empty_mask_is_background_bit_exact(tiny):
    codes = np.zeros_like(tiny.codes[:2])
    r = oracle.render(tiny.scene, tiny.camera, tiny.basis, codes, BG)
    assert np.all(r["image"] == BG.astype(np.float64)[None, None, None, :])
    assert np.all(r["tfinal"] == 1.0)


def test_full_mask_equals_unmasked_bit_exact():
    w = synth.make_workload("g250k_800px_64states", n=3000, states=2)
    cam = synth.ring_camera(64, 64)
    full = np.full((1, w.scene.num_packets), 4, np.uint8)
    pix = np.stack(np.meshgrid(np.arange(0, 64, 3), np.arange(0, 64, 3)), -1).reshape(-1, 2)
    r1 = oracle.render(w.scene, cam, w.basis, full, BG, pixels=pix)
    flat = replace(w.scene, packet_layer=(w.scene.packet_layer & np.uint16(0xFFFC)))
    r2 = oracle.render(flat, cam, w.basis, np.ones_like(full), BG, pixels=pix)
    assert np.array_equal(r1["image"], r2["image"])


def test_prefix_monotone_coverage():
    w = synth.make_workload("g250k_800px_64states", n=4000, states=6)
    cam = synth.ring_camera(48, 48)
    codes = w.codes.copy()
    deeper = np.minimum(codes.astype(np.int64) + 1, 4).astype(np.uint8)
    for k in range(codes.shape[0]):
        p0 = oracle.present_mask(w.scene, codes[k])
        p1 = oracle.present_mask(w.scene, deeper[k])
        assert np.all(p1[p0])  # present set grows with the prefix depth
    r0 = oracle.render(w.scene, cam, w.basis, codes, BG)
    r1 = oracle.render(w.scene, cam, w.basis, deeper, BG)
    assert np.all(r1["tfinal"] <= r0["tfinal"] + 1e-4)  # include-then-stop bound


def test_transmittance_range(tiny):
    r = oracle.render(tiny.scene, tiny.camera, tiny.basis, tiny.codes[:4], BG)
    T = r["tfinal"]
    assert np.all(T > 0) and np.all(T <= 1)
    assert np.array_equal(T == 1.0, r["ncomp"] == 0)


# ----------------------------------------------- P8 independent FP64 twin

def test_dense_twin_matches_per_pixel_oracle(tiny):
    import oracle.grad as og
    rng = np.random.default_rng(3)
    pix = rng.integers(0, 128, size=(300, 2))
    r = oracle.render(tiny.scene, tiny.camera, tiny.basis, tiny.codes, BG, pixels=pix)
    img, _ = og.render_dense(tiny.scene, tiny.camera, tiny.basis, tiny.codes, BG, pixels=pix)
    np.testing.assert_allclose(img.detach().numpy(), r["image"], rtol=0, atol=1e-12)


# -------------------------------------------------- P9 binning and order

@pytest.mark.parametrize("tw,th", [(16, 16), (32, 8)])
def test_tile_rect_is_conservative(tiny, tw, th):
    """Every pixel where a Gaussian reaches alpha >= 1/255 (FP64) lies in a
    tile of that Gaussian's FP32 rectangle: binning never changes an image."""
    sc, cam = tiny.scene, tiny.camera
    m = oracle.mirror_f32(sc, cam, tiny.basis, tw, th)
    g = oracle.geometry_f64(sc, cam, tiny.basis)
    ys, xs = np.meshgrid(np.arange(cam.height) + 0.5, np.arange(cam.width) + 0.5, indexing="ij")
    xs, ys = xs.reshape(-1), ys.reshape(-1)
    tx, ty = (xs // tw).astype(np.int64), (ys // th).astype(np.int64)
    bad = 0
    for i0 in range(0, sc.n, 256):
        sl = slice(i0, i0 + 256)
        dx = g["u"][sl, None] - xs[None]
        dy = g["v"][sl, None] - ys[None]
        q = g["conA"][sl, None] * dx * dx + 2 * g["conB"][sl, None] * dx * dy + g["conC"][sl, None] * dy * dy
        al = np.minimum(0.99, g["o"][sl, None] * np.exp(-0.5 * q))
        hit = (al >= 1 / 255) & m["valid"][sl, None]
        r = m["rect"][:, sl]
        inside = (tx[None] >= r[0][:, None]) & (tx[None] < r[2][:, None]) & \
                 (ty[None] >= r[1][:, None]) & (ty[None] < r[3][:, None])
        bad += int(np.count_nonzero(hit & ~inside))
    assert bad == 0


def test_tile_lists_equal_brute_force_sort():
    sc = overlap_scene(n=40, spread=0.6, log_scale=-2.0)
    cam = synth.ring_camera(64, 48)
    m = oracle.mirror_f32(sc, cam, BASIS0, 16, 16)
    ranges, ids, keys = oracle.tile_lists(m, 64, 48)
    tiles_x = 4
    for t in range(ranges.shape[0]):
        tx, ty = t % tiles_x, t // tiles_x
        want = sorted((int(m["zbits"][i]), i) for i in range(sc.n)
                      if m["valid"][i] and m["rect"][0, i] <= tx < m["rect"][2, i]
                      and m["rect"][1, i] <= ty < m["rect"][3, i])
        got = ids[ranges[t, 0]:ranges[t, 1]].tolist()
        assert got == [i for _, i in want]
        assert np.all(keys[ranges[t, 0]:ranges[t, 1]] >> np.uint64(32) == t)


def test_mirror_close_to_fp64(tiny):
    m = oracle.mirror_f32(tiny.scene, tiny.camera, tiny.basis)
    g = oracle.geometry_f64(tiny.scene, tiny.camera, tiny.basis)
    assert np.max(np.abs(m["z32"] / g["Z"] - 1)) < 1e-6
    for k in ("a", "c"):
        assert np.max(np.abs(m[k] / g[k] - 1)) < 2e-5
    assert np.max(np.abs(m["u"] - g["u"])) < 1e-4 and np.max(np.abs(m["v"] - g["v"])) < 1e-4
    assert np.array_equal(m["valid"], g["Z"] > tiny.camera.near)


def test_near_plane_culls():
    sc = scene_from_lists([[0, 0, -3.5], [0, 0, -2.995], [0, 0, 0.0]], [math.log(0.1)] * 3)
    cam = synth.ring_camera(32, 32)
    m = oracle.mirror_f32(sc, cam, BASIS0)
    assert m["valid"].tolist() == [False, False, True]  # z = -0.5, 0.005 <= near, 3
    r = oracle.render(sc, cam, BASIS0, np.ones((1, 1), np.uint8), BG)
    assert r["ncomp"].max() == 1


# ------------------------------------- Eq. (1) deformation, affine, rotation

def test_temporal_deformation_closed_form():
    rng = np.random.default_rng(5)
    tc = rng.normal(0, 0.1, size=(3, 6))
    sc = scene_from_lists(rng.uniform(-0.5, 0.5, (3, 3)), [math.log(0.1)] * 3, temporal=tc)
    cam = synth.ring_camera(32, 32)
    basis = np.array([0.5, 0.25], np.float32)
    g = oracle.geometry_f64(sc, cam, basis)
    for i in range(3):
        mu = sc.mean[:, i].astype(np.float64) + basis[0] * sc.temporal[0:3, i].astype(np.float64) \
            + basis[1] * sc.temporal[3:6, i].astype(np.float64)
        P = cam.R_cw.astype(np.float64) @ mu + cam.t_cw
        assert np.allclose([g["X"][i], g["Y"][i], g["Z"][i]], P, rtol=0, atol=1e-14)
    # b(t) = 0 (t = 0): the temporal coefficients have no effect
    g0 = oracle.geometry_f64(sc, cam, BASIS0)
    g1 = oracle.geometry_f64(replace(sc, temporal=np.zeros_like(sc.temporal)), cam, BASIS0)
    for k in g0:
        assert np.array_equal(g0[k], g1[k])


def test_cluster_affine():
    rng = np.random.default_rng(6)
    sc = scene_from_lists(rng.uniform(-0.5, 0.5, (4, 3)), [math.log(0.1)] * 3,
                          packet_layer=np.array([0, 0, 4, 4]), clusters=2, contexts=1,
                          temporal=rng.normal(0, 0.05, (4, 6)))
    cam = synth.ring_camera(32, 32)
    basis = np.array([0.5, 0.25], np.float32)
    ident = np.tile(np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32), (2, 1))
    a0 = oracle.geometry_f64(sc, cam, basis)
    a1 = oracle.geometry_f64(replace(sc, cluster_affine=ident), cam, basis)
    for k in a0:
        assert np.array_equal(a0[k], a1[k])
    m0 = oracle.mirror_f32(sc, cam, basis)
    m1 = oracle.mirror_f32(replace(sc, cluster_affine=ident), cam, basis)
    for k in ("z32", "u", "v", "a", "b", "c"):
        assert np.array_equal(m0[k], m1[k])
    # cluster 1 translated by d: its camera-frame means move by R_cw d
    aff = ident.copy()
    d = np.array([0.1, -0.2, 0.05], np.float32)
    aff[1, [3, 7, 11]] = d
    a2 = oracle.geometry_f64(replace(sc, cluster_affine=aff), cam, basis)
    mv = cam.R_cw.astype(np.float64) @ d.astype(np.float64)
    for i in range(4):
        shift = mv if i >= 2 else 0.0
        got = np.array([a2["X"][i], a2["Y"][i], a2["Z"][i]])
        ref = np.array([a0["X"][i], a0["Y"][i], a0["Z"][i]]) + shift
        assert np.allclose(got, ref, atol=1e-14)


def test_quaternion_invariances():
    rng = np.random.default_rng(8)
    q = rng.normal(size=(1, 4))
    ls = [[math.log(0.05), math.log(0.12), math.log(0.08)]]
    cam = synth.ring_camera(64, 64)
    base = oracle.geometry_f64(scene_from_lists([[0.1, 0.2, 0.3]], ls, q), cam, BASIS0)
    for qq in (-q, 2.5 * q):
        g = oracle.geometry_f64(scene_from_lists([[0.1, 0.2, 0.3]], ls, qq), cam, BASIS0)
        for k in ("a", "b", "c"):  # 2.5 q is rounded to FP32 on input
            assert g[k][0] == pytest.approx(base[k][0], rel=1e-5)
    # isotropic scale: covariance independent of the rotation
    iso = [[math.log(0.1)] * 3]
    g0 = oracle.geometry_f64(scene_from_lists([[0, 0, 0]], iso, [[1, 0, 0, 0]]), cam, BASIS0)
    g1 = oracle.geometry_f64(scene_from_lists([[0, 0, 0]], iso, q), cam, BASIS0)
    for k in ("a", "b", "c"):
        assert g1[k][0] == pytest.approx(g0[k][0], rel=1e-12, abs=1e-12)
    # 90 degrees about the viewing axis (world z for this camera) swaps a and c
    ls2 = [[math.log(0.05), math.log(0.15), math.log(0.1)]]
    h = math.sqrt(0.5)
    ga = oracle.geometry_f64(scene_from_lists([[0, 0, 0]], ls2, [[1, 0, 0, 0]]), cam, BASIS0)
    gb = oracle.geometry_f64(scene_from_lists([[0, 0, 0]], ls2, [[h, 0, 0, h]]), cam, BASIS0)
    assert gb["a"][0] == pytest.approx(ga["c"][0], rel=1e-6)
    assert gb["c"][0] == pytest.approx(ga["a"][0], rel=1e-6)
    assert ga["a"][0] < ga["c"][0]


def test_sh1_colour_closed_form():
    C0 = 1.0 / (2.0 * math.sqrt(math.pi))
    C1 = math.sqrt(3.0) / (2.0 * math.sqrt(math.pi))
    cam = synth.ring_camera(32, 32)  # centre (0, 0, -3)
    col = np.zeros(12)
    col[0:3] = [0.3, -0.2, 0.1]       # DC
    col[6:9] = [0.2, 0.4, -0.9]      # z coefficient (k2)
    sc = scene_from_lists([[0, 0, 0]], [math.log(0.1)] * 3, colors=[col], sh_degree=1)
    g = oracle.geometry_f64(sc, cam, BASIS0)
    k = sc.color[:, 0].astype(np.float64).reshape(4, 3)
    exp = np.maximum(0.0, 0.5 + C0 * k[0] + C1 * k[2])  # direction (0, 0, 1)
    assert np.allclose([g["r"][0], g["g"][0], g["b_"][0]], exp, atol=1e-15)
    # y-offset Gaussian: only the y coefficient (k1) with the -d_y sign
    col = np.zeros(12)
    col[3:6] = [0.5, -0.5, 0.25]
    sc = scene_from_lists([[0, 0.6, 0]], [math.log(0.1)] * 3, colors=[col], sh_degree=1)
    g = oracle.geometry_f64(sc, cam, BASIS0)
    d = np.array([0.0, float(np.float32(0.6)), 3.0])
    d /= np.linalg.norm(d)
    k = sc.color[:, 0].astype(np.float64).reshape(4, 3)
    exp = np.maximum(0.0, 0.5 - C1 * d[1] * k[1])
    assert np.allclose([g["r"][0], g["g"][0], g["b_"][0]], exp, atol=1e-15)


# ------------------------------------------------------------ P12 gradients

def _fd_check(sc, cam, basis, codes, gimg, idxs, rel=1e-6):
    import torch

    import oracle.grad as og
    ref = og.gradients(sc, cam, basis, codes, BG, gimg)
    gi = torch.as_tensor(gimg.reshape(codes.shape[0], -1, 3))
    checked = 0
    for name in og.PARAMS:
        base = og.params_from_scene(sc, requires_grad=False)
        arr = base[name]
        flat = arr.reshape(-1, arr.shape[-1])
        for row in range(flat.shape[0]):
            for i in idxs:
                v0 = float(flat[row, i])
                h = 1e-6 * max(1.0, abs(v0))
                vals = []
                for sgn in (1, -1):
                    p = {k: t.clone() for k, t in base.items()}
                    p[name].reshape(-1, arr.shape[-1])[row, i] = v0 + sgn * h
                    img, _ = og.render_dense(sc, cam, basis, codes, BG, params=p)
                    vals.append(float((img * gi).sum()))
                fd = (vals[0] - vals[1]) / (2 * h)
                an = ref[name].reshape(-1, arr.shape[-1])[row, i]
                assert abs(fd - an) <= rel * max(1.0, abs(an)) + 1e-8, (name, row, i, fd, an)
                checked += 1
    return ref, checked


def test_gradient_matches_central_differences():
    sc = overlap_scene(n=8, spread=0.25, log_scale=-1.3)
    cam = synth.ring_camera(24, 24)
    basis = np.array([0.5, 0.25], np.float32)
    rng = np.random.default_rng(11)
    codes = rng.integers(0, 5, size=(3, sc.num_packets)).astype(np.uint8)
    codes[0] = 4
    gimg = rng.normal(size=(3, 24, 24, 3))
    ref, checked = _fd_check(sc, cam, basis, codes, gimg, idxs=range(8))
    assert checked == 8 * (3 + 3 + 4 + 1 + 12 + 6)
    assert all(np.any(ref[k] != 0) for k in ref)


def test_gradient_special_cases():
    import oracle.grad as og
    sc = overlap_scene(n=6, spread=0.2, log_scale=-1.3)
    cam = synth.ring_camera(24, 24)
    codes = np.full((2, sc.num_packets), 4, np.uint8)
    gimg = np.random.default_rng(2).normal(size=(2, 24, 24, 3))
    g = og.gradients(sc, cam, BASIS0, codes, BG, gimg)
    assert np.all(g["temporal"] == 0.0)  # b(t) = 0
    iso = replace(sc, log_scale=np.repeat(sc.log_scale[:1], 3, axis=0))
    g = og.gradients(iso, cam, BASIS0, codes, BG, gimg)
    assert np.max(np.abs(g["quat"])) <= 1e-10 * np.max(np.abs(g["mean"]))


# ---------------------------------------------------------------- PSNR

def test_psnr_definition():
    ref = np.full((4, 5, 3), 0.5)
    img = np.stack([ref, ref + 0.1, ref - 0.01])
    p = oracle.psnr(img, ref)
    assert p[0] == pytest.approx(100.0)
    assert p[1] == pytest.approx(20.0)
    assert p[2] == pytest.approx(40.0)


def test_l1_loss_and_gradient():
    """Plain L1 loss: a hand-computed value, sign(0) = 0 in the gradient, and
    the gradient against central differences of the value away from ties."""
    import oracle.grad as og
    img = np.array([[[[0.5, 0.25, 1.0]], [[0.0, 0.75, 0.5]]]])  # [1, 2, 1, 3]
    tgt = np.array([[[[0.25, 0.25, 0.0]], [[0.5, 0.5, 0.5]]]])
    # |d| = 0.25, 0, 1, 0.5, 0.25, 0 -> mean 2 / 6
    assert og.l1_loss(img, tgt) == pytest.approx(2.0 / 6.0, abs=1e-15)
    g = og.l1_loss_grad(img, tgt)
    assert np.array_equal(g.reshape(-1) * 6, [1, 0, 1, -1, 1, 0])
    rng = np.random.default_rng(2)
    x, t = rng.uniform(0, 1, (3, 4, 5, 3)), rng.uniform(0, 1, (1, 4, 5, 3))
    g = og.l1_loss_grad(x, t)
    h = 1e-7
    for idx in [(0, 0, 0, 0), (1, 2, 3, 1), (2, 3, 4, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (og.l1_loss(xp, t) - og.l1_loss(xm, t)) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6)


# --------------------------------------------------------- stored fixtures

def test_golden_oracle_regression():
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(here, "oracle_tiny.json")) as f:
        gold = json.load(f)
    w = synth.make_workload(gold["workload"], background=gold["background"])
    r = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background,
                      pixels=np.array(gold["pixels"]))
    np.testing.assert_allclose(r["image"], np.array(gold["image"]), rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["tfinal"], np.array(gold["tfinal"]), rtol=0, atol=1e-12)


def test_workloads_follow_paper_structure():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_structure.json")) as f:
        ps = json.load(f)
    for name, rec in synth.WORKLOADS.items():
        assert rec["layers"] in (1, ps["layers_per_cluster"]["value"])
    w = synth.make_workload("g250k_800px_64states", n=2000, states=3)
    assert w.scene.rank == ps["temporal_rank"]["value"]
    assert int((w.scene.packet_layer & 3).max()) == ps["layers_per_cluster"]["value"] - 1
