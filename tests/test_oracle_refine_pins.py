"""Pins for the oracle's attribute-level prefix refinement (Sec. 3: position by
Eq. (1) plus residual levels; scale, rotation, opacity and colour as a base
plus three refinements; one base and three refinement groups per cluster).

Each check is a closed form for one or two Gaussians seen by the theta = 0
ring camera (camera x = -world x, y = -world y, z = world z + 3), written
from the projection's mathematics, or a special case that reduces to the
plain renderer.  A refinement level applied at the wrong depth, a sign, a
residual added before the affine deformation, or a dropped rotation or
colour level each fails one of them.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from tests.scenes_for_tests import logit, scene_from_lists

BG = np.array([0.25, 0.5, 0.75], np.float32)
BG64 = BG.astype(np.float64)
SH_C0 = 0.5 / math.sqrt(math.pi)
SH_C1 = math.sqrt(3.0) / (2.0 * math.sqrt(math.pi))


def _levels(n, sh_degree=0):
    return np.zeros((3, oracle.refine_rows(sh_degree), n), np.float32)


def _sig(x):
    return 1.0 / (1.0 + math.exp(-x))


def _closed_form(cam, gs, bg=BG64):
    """Image of Gaussians with camera-frame mean (X, 0, Z) and camera-axis
    variances (vx, vy, vz): u = fx X/Z + cx, v = cy; 2D covariance
    diag((fx/Z)^2 vx + (fx X/Z^2)^2 vz + 0.3, (fy/Z)^2 vy + 0.3); alpha =
    min(0.99, o exp(-q/2)) kept when >= 1/255; front to back by Z."""
    H, Wd = cam.height, cam.width
    img = np.zeros((H, Wd, 3))
    fx, fy = float(cam.fx), float(cam.fy)
    order = sorted(gs, key=lambda g: g["Z"])
    for py in range(H):
        for px in range(Wd):
            T, C = 1.0, np.zeros(3)
            for g in order:
                X, Z = g["X"], g["Z"]
                a = (fx / Z) ** 2 * g["vx"] + (fx * X / Z ** 2) ** 2 * g["vz"] + 0.3
                c = (fy / Z) ** 2 * g["vy"] + 0.3
                dx = px + 0.5 - (fx * X / Z + cam.cx)
                dy = py + 0.5 - cam.cy
                al = min(0.99, g["o"] * math.exp(-0.5 * (dx * dx / a + dy * dy / c)))
                if al < 1.0 / 255.0:
                    continue
                C += T * al * np.asarray(g["col"], np.float64)
                T *= 1.0 - al
            img[py, px] = C + T * bg
    return img


def test_levels_apply_by_delivered_depth_closed_form():
    """One Gaussian, opacity / colour / scale / x-residual refined per level;
    every code 0..5 against the closed form (codes above 4 act as 4)."""
    m = (0.05, 0.0, 0.2)
    s0, l0, c0 = math.log(0.06), logit(0.5), [0.3, 0.5, 0.7]
    q_t = [[0.1, 0.0, 0.0, 0.02, 0.0, 0.0]]  # temporal coefficients: x moves with b_0 and b_1
    sc = scene_from_lists([m], [s0] * 3, None, [l0], [c0], q_t, rank=2)
    basis = np.array([0.5, -0.25], np.float32)
    ref = _levels(1)
    dx = [0.03, -0.05, 0.02]
    ds = [0.2, -0.1, 0.15]
    dl = [1.0, -0.5, 0.8]
    dc = [[0.1, -0.2, 0.05], [0.02, 0.1, -0.1], [-0.05, 0.03, 0.2]]
    for j in range(3):
        ref[j, 0, 0] = dx[j]
        ref[j, 3:6, 0] = ds[j]
        ref[j, 10, 0] = dl[j]
        ref[j, 11:14, 0] = dc[j]
    cam = synth.ring_camera(40, 24)
    codes = np.arange(6, dtype=np.uint8).reshape(6, 1)
    r = oracle.render_refined(sc, ref, cam, basis, codes, BG)
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    for c in range(6):
        if c == 0:
            want = np.broadcast_to(BG64, (24, 40, 3))
        else:
            d = min(c, 4) - 1
            x = f32(m[0]) + 0.5 * f32(0.1) - 0.25 * f32(0.02) + sum(f32(v) for v in dx[:d])
            sl = f32(s0) + sum(f32(v) for v in ds[:d])
            var = math.exp(2 * sl)
            o = _sig(f32(l0) + sum(f32(v) for v in dl[:d]))
            col = np.array([f32(v) for v in c0]) + sum(np.array([f32(v) for v in dc[j]]) for j in range(d))
            want = _closed_form(cam, [dict(X=-x, Z=f32(m[2]) + 3.0, vx=var, vy=var, vz=var, o=o, col=col)])
        np.testing.assert_allclose(r["image"][c], want, rtol=0, atol=2e-6, err_msg=f"code {c}")
    # each level changes the image
    for c in range(1, 4):
        assert np.abs(r["image"][c + 1] - r["image"][c]).max() > 1e-3


def test_rotation_levels_turn_the_covariance():
    """Anisotropic Gaussian on the axis: level 1 adds (0,0,0,1) to the
    quaternion (1,0,0,0) -> a quarter turn about z swaps the x and y
    variances; level 2 adds (0,0,0,-1) and undoes it; level 3 adds
    (0.5,0,0,0), which normalisation removes."""
    sx, sy, sz = 0.03, 0.09, 0.05
    sc = scene_from_lists([[0.0, 0.0, 0.0]], [[math.log(sx), math.log(sy), math.log(sz)]], None,
                          [logit(0.8)], [[0.9, 0.1, 0.3]])
    ref = _levels(1)
    ref[0, 9, 0] = 1.0
    ref[1, 9, 0] = -1.0
    ref[2, 6, 0] = 0.5
    cam = synth.ring_camera(32, 32)
    codes = np.array([[1], [2], [3], [4]], np.uint8)
    r = oracle.render_refined(sc, ref, cam, np.zeros(2, np.float32), codes, BG)
    v = [math.exp(2 * float(np.float32(math.log(s)))) for s in (sx, sy, sz)]
    col = np.array([float(np.float32(c)) for c in (0.9, 0.1, 0.3)])
    o = _sig(float(np.float32(logit(0.8))))
    plain = _closed_form(cam, [dict(X=0.0, Z=3.0, vx=v[0], vy=v[1], vz=v[2], o=o, col=col)])
    turned = _closed_form(cam, [dict(X=0.0, Z=3.0, vx=v[1], vy=v[0], vz=v[2], o=o, col=col)])
    assert np.abs(plain - turned).max() > 0.05
    for k, want in enumerate([plain, turned, plain, plain]):
        np.testing.assert_allclose(r["image"][k], want, rtol=0, atol=1e-6, err_msg=f"code {k + 1}")


def test_layers_and_packets_take_their_own_depth():
    """Two packets: A (packet 0, layer 0) in front, B (packet 1, layer 2)
    behind; B is absent below code 3, and each takes its own packet's depth."""
    sA, sB = math.log(0.05), math.log(0.07)
    sc = scene_from_lists([[-0.1, 0.0, 0.0], [0.12, 0.0, 0.4]], [[sA] * 3, [sB] * 3], None,
                          [logit(0.6), logit(0.7)], [[0.8, 0.2, 0.1], [0.1, 0.3, 0.9]],
                          packet_layer=[(0 << 2) | 0, (1 << 2) | 2], clusters=1, contexts=2)
    ref = _levels(2)
    dl = np.array([[0.4, -0.3], [-0.6, 0.9], [0.2, 0.5]], np.float32)  # [level][gaussian]
    dsc = np.array([[0.1, 0.2], [0.3, -0.2], [-0.1, 0.25]], np.float32)
    ref[:, 10, :] = dl
    ref[:, 3:6, :] = dsc[:, None, :]
    cam = synth.ring_camera(48, 24)
    codes = np.array([[1, 2], [3, 3], [0, 4], [2, 7], [4, 1]], np.uint8)
    r = oracle.render_refined(sc, ref, cam, np.zeros(2, np.float32), codes, BG)
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    base_s, base_l = [f32(sA), f32(sB)], [f32(logit(0.6)), f32(logit(0.7))]
    X = [-f32(-0.1), -f32(0.12)]
    Z = [3.0, f32(0.4) + 3.0]
    cols = [np.array([f32(c) for c in (0.8, 0.2, 0.1)]), np.array([f32(c) for c in (0.1, 0.3, 0.9)])]
    layer = [0, 2]
    for k, row in enumerate(codes):
        gs = []
        for i in range(2):
            code = int(row[i])
            if layer[i] >= code:
                continue
            d = min(code, 4) - 1
            s = base_s[i] + float(dsc[:d, i].astype(np.float64).sum())
            lg = base_l[i] + float(dl[:d, i].astype(np.float64).sum())
            var = math.exp(2 * s)
            gs.append(dict(X=X[i], Z=Z[i], vx=var, vy=var, vz=var, o=_sig(lg), col=cols[i]))
        np.testing.assert_allclose(r["image"][k], _closed_form(cam, gs), rtol=0, atol=2e-6,
                                   err_msg=f"codes {row}")


def test_position_residual_follows_the_affine_deformation():
    """Cluster affine A = 2 I with translation (0.1, 0, 0.2): the mean is
    A [mubar; 1] + b q + o, so u = fx X / Z + cx with X = -(2 m_x + 0.1 +
    b q_x + o_x); adding o before the affine would double it."""
    aff = np.array([[2, 0, 0, 0.1, 0, 2, 0, 0, 0, 0, 2, 0.2]], np.float32)
    sc = scene_from_lists([[0.04, 0.0, 0.1]], [math.log(0.05)] * 3, None, [logit(0.5)], [[0.5, 0.5, 0.5]],
                          [[0.2, 0.0, 0.0, 0.0, 0.0, 0.0]], rank=2, cluster_affine=aff)
    basis = np.array([0.3, 0.0], np.float32)
    ref = _levels(1)
    ref[:, 0, 0] = [0.05, -0.02, 0.0]
    ref[:, 2, 0] = [0.1, 0.05, 0.0]
    cam = synth.ring_camera(64, 64)
    f = float(cam.fx)
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    for code in (1, 2, 3, 4):
        d = code - 1
        g = oracle.geometry_f64(oracle.refined_scene(sc, ref, np.array([code], np.uint8)), cam, basis)
        x = 2 * f32(0.04) + f32(0.1) + f32(0.3) * f32(0.2) + sum(f32(v) for v in [0.05, -0.02, 0.0][:d])
        z = 2 * f32(0.1) + f32(0.2) + sum(f32(v) for v in [0.1, 0.05, 0.0][:d])
        assert g["X"][0] == pytest.approx(-x, abs=1e-7)
        assert g["Z"][0] == pytest.approx(z + 3.0, abs=1e-7)
        assert g["u"][0] == pytest.approx(f * (-x) / (z + 3.0) + cam.cx, abs=1e-4)


def test_sh_colour_levels_on_the_axis():
    """Degree-1 SH seen along +z: colour = 0.5 + C0 k0 + C1 k2 per channel
    (the x and y direction terms vanish); levels add to k0 and k2 and leave
    k1, k3 without effect."""
    k = np.zeros(12)
    k[0:3] = [0.2, -0.1, 0.4]    # k0 per channel
    k[3:6] = [0.7, 0.7, 0.7]     # k1 (x direction: no effect)
    k[6:9] = [0.1, 0.3, -0.2]    # k2 (z direction)
    k[9:12] = [-0.9, 0.5, 0.2]   # k3 (no effect)
    sc = scene_from_lists([[0.0, 0.0, 0.0]], [math.log(0.05)] * 3, None, [logit(0.5)], [k], sh_degree=1)
    ref = _levels(1, sh_degree=1)
    lv = np.array([[0.05, 0.1, -0.1, 0.02, -0.03, 0.04],
                   [-0.02, 0.01, 0.03, 0.1, 0.0, -0.05],
                   [0.01, -0.04, 0.02, -0.01, 0.05, 0.03]], np.float32)  # [level][k0 rgb, k2 rgb]
    ref[:, 11:14, 0] = lv[:, :3]
    ref[:, 17:20, 0] = lv[:, 3:]
    ref[:, 14:17, 0] = 5.0   # k1 levels: no effect on the axis
    ref[:, 20:23, 0] = -5.0  # k3 levels: likewise
    cam = synth.ring_camera(16, 16)
    k32 = k.astype(np.float32).astype(np.float64)
    for code in (1, 2, 3, 4):
        d = code - 1
        g = oracle.geometry_f64(oracle.refined_scene(sc, ref, np.array([code], np.uint8)), cam, np.zeros(2, np.float32))
        k0 = k32[0:3] + lv[:d, :3].astype(np.float64).sum(axis=0)
        k2 = k32[6:9] + lv[:d, 3:].astype(np.float64).sum(axis=0)
        want = np.maximum(0.5 + SH_C0 * k0 + SH_C1 * k2, 0.0)
        got = np.array([g["r"][0], g["g"][0], g["b_"][0]])
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-7, err_msg=f"code {code}")


def test_zero_levels_and_base_only_states_reduce_to_the_plain_renderer():
    """All-zero levels leave every state's render unchanged (bit for bit);
    with non-zero levels, states whose codes are 0 or 1 use none of them."""
    sc = synth.make_scene(400, 4, 2, 4, "sh1", index=21, stream=0)
    cam = synth.ring_camera(48, 40)
    basis = synth.temporal_basis(0.3, sc.rank)
    codes = synth.make_codes("present_depth", 0.3, 0.9, 5, sc.num_packets, 4, index=21)
    plain = oracle.render(sc, cam, basis, codes, BG)
    zero = oracle.render_refined(sc, np.zeros((3, oracle.refine_rows(1), sc.n), np.float32), cam, basis, codes, BG)
    for key in ("image", "tfinal", "ncomp"):
        np.testing.assert_array_equal(zero[key], plain[key])
    levels = synth.make_refinement(sc, index=21)
    base_codes = np.minimum(codes, 1)
    a = oracle.render_refined(sc, levels, cam, basis, base_codes, BG)
    b = oracle.render(sc, cam, basis, base_codes, BG)
    np.testing.assert_array_equal(a["image"], b["image"])
    # and the levels do change full-depth states
    full = np.full((1, sc.num_packets), 4, np.uint8)
    c = oracle.render_refined(sc, levels, cam, basis, full, BG)["image"]
    assert np.abs(c - oracle.render(sc, cam, basis, full, BG)["image"]).max() > 1e-3


def test_refinement_generator_shapes_and_scales():
    sc = synth.make_scene(2000, 4, 2, 4, "rgb", index=3, stream=0)
    lv = synth.make_refinement(sc, index=3)
    assert lv.shape == (3, oracle.refine_rows(0), sc.n) and lv.dtype == np.float32
    assert np.all(lv[2, :3] == 0.0)  # no position residual on the last level
    for j in range(3):
        assert lv[j, 10].std() == pytest.approx(0.5 * 2.0 ** -j, rel=0.1)
    assert np.array_equal(lv, synth.make_refinement(sc, index=3))


# ------------------------------------------------------------- gradients
def _grad_case(n=24, seed=3):
    import oracle.grad as og  # noqa: F401
    from tests.scenes_for_tests import overlap_scene
    sc = overlap_scene(n=n, seed=seed, sh_degree=1, rank=2)
    cam = synth.ring_camera(24, 20)
    basis = np.array([0.5, 0.25], np.float32)
    rng = np.random.default_rng(seed)
    lv = (rng.normal(0, 1, (3, oracle.refine_rows(1), n)) *
          np.array([0.01] * 3 + [0.1] * 3 + [0.1] * 4 + [0.5] + [0.05] * 12)[None, :, None]).astype(np.float32)
    codes = np.array([[1, 2, 3, 4], [4, 4, 4, 4], [0, 3, 2, 1], [2, 0, 4, 3]], np.uint8)
    return sc, cam, basis, lv, codes


def test_dense_refined_forward_matches_the_per_state_decode():
    """The differentiable FP64 formulation (attribute sums in FP64, alphas in
    dense rows) against the C renderer of each decoded state (FP32 sums)."""
    import oracle.grad as og
    sc, cam, basis, lv, codes = _grad_case()
    dense = og.render_dense_refined(sc, lv, cam, basis, codes, BG).detach().numpy()
    ref = oracle.render_refined(sc, lv, cam, basis, codes, BG)
    d = np.abs(dense.reshape(ref["image"].shape) - ref["image"]).max(-1) - ref["budget"]
    assert d.max() <= 2e-6, d.max()


def test_refined_gradients_match_central_differences():
    import torch
    import oracle.grad as og
    sc, cam, basis, lv, codes = _grad_case()
    rng = np.random.default_rng(1)
    gi = rng.normal(size=(codes.shape[0], cam.height * cam.width, 3))
    g = og.gradients_refined(sc, lv, cam, basis, codes, BG, gi)
    base = og.params_from_scene(sc, requires_grad=False)
    lvt = torch.tensor(lv.astype(np.float64))

    def f(b, l):
        return float((og.render_dense_refined(sc, lv, cam, basis, codes, BG, None, b, l) * torch.as_tensor(gi)).sum())

    h = 1e-6
    picks = [("refine", (j, r, i)) for j in range(3) for r in (0, 2, 4, 7, 10, 13) for i in (0, 5, 11)]
    picks += [(k, idx) for k, idx in (("mean", (0, 3)), ("log_scale", (1, 7)), ("quat", (2, 9)),
                                      ("opacity_logit", (4,)), ("color", (5, 2)), ("temporal", (3, 6)))]
    checked = 0
    for k, idx in picks:
        if k == "refine":
            lp, lm = lvt.clone(), lvt.clone()
            lp[idx] += h
            lm[idx] -= h
            fd = (f(base, lp) - f(base, lm)) / (2 * h)
        else:
            bp = {kk: v.clone() for kk, v in base.items()}
            bm = {kk: v.clone() for kk, v in base.items()}
            bp[k][idx] += h
            bm[k][idx] -= h
            fd = (f(bp, lvt) - f(bm, lvt)) / (2 * h)
        assert g[k][idx] == pytest.approx(fd, abs=1e-6, rel=1e-5), (k, idx, g[k][idx], fd)
        checked += abs(fd) > 1e-4
    assert checked >= 10  # the picks exercise real gradients


def test_refined_gradients_of_base_only_states():
    """States delivering depth 0 everywhere use no level: the level gradients
    are exactly zero and the base gradients are the plain renderer's."""
    import oracle.grad as og
    sc, cam, basis, lv, _ = _grad_case()
    codes = np.array([[1, 1, 1, 1], [1, 0, 1, 1]], np.uint8)
    rng = np.random.default_rng(2)
    gi = rng.normal(size=(2, cam.height * cam.width, 3))
    g = og.gradients_refined(sc, lv, cam, basis, codes, BG, gi)
    assert np.all(g["refine"] == 0.0)
    plain = og.gradients(sc, cam, basis, codes, BG, gi)
    for k in og.PARAMS:
        np.testing.assert_allclose(g[k], plain[k], rtol=0, atol=1e-12, err_msg=k)
