"""Property checks of the oracle on generated tiny scenes (off-screen and
culled Gaussians, sub-pixel and elongated footprints, depth ties, cluster
affines, codes above 4): the per-pixel C oracle and the independent dense
PyTorch FP64 twin agree at every pixel (P8: binning-free definitions); tile
rectangles are conservative (every pixel where a Gaussian reaches 1/255 is
inside its rectangle); tile lists equal a brute-force sort."""

import numpy as np
from hypothesis import HealthCheck, given, settings

import oracle
import oracle.grad as og
from tests.hyp_scenes import tiny_scenes

BG = np.array([0.25, 0.5, 0.75], np.float32)
SETTINGS = dict(max_examples=40, deadline=None, derandomize=True,
                suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


@settings(**SETTINGS)
@given(tiny_scenes())
def test_dense_twin_equals_per_pixel_oracle(case):
    scene, cam, basis, codes = case
    r = oracle.render(scene, cam, basis, codes, BG)
    img, _ = og.render_dense(scene, cam, basis, codes, BG)
    H, Wd = cam.height, cam.width
    np.testing.assert_allclose(img.detach().numpy().reshape(codes.shape[0], H, Wd, 3), r["image"], rtol=0,
                               atol=1e-12)
    assert np.all(r["tfinal"] > 0) and np.all(r["tfinal"] <= 1)


@settings(**SETTINGS)
@given(tiny_scenes())
def test_rectangles_conservative_and_lists_sorted(case):
    scene, cam, basis, _ = case
    g = oracle.geometry_f64(scene, cam, basis)
    for tw, th in ((16, 16), (32, 8)):
        m = oracle.mirror_f32(scene, cam, basis, tw, th)
        ys, xs = np.meshgrid(np.arange(cam.height) + 0.5, np.arange(cam.width) + 0.5, indexing="ij")
        xs, ys = xs.reshape(-1), ys.reshape(-1)
        dx = g["u"][:, None] - xs[None]
        dy = g["v"][:, None] - ys[None]
        q = g["conA"][:, None] * dx * dx + 2 * g["conB"][:, None] * dx * dy + g["conC"][:, None] * dy * dy
        hit = (np.minimum(0.99, g["o"][:, None] * np.exp(-0.5 * q)) >= 1 / 255) & m["valid"][:, None]
        r = m["rect"]
        tx, ty = (xs // tw).astype(np.int64), (ys // th).astype(np.int64)
        inside = (tx[None] >= r[0][:, None]) & (tx[None] < r[2][:, None]) & \
                 (ty[None] >= r[1][:, None]) & (ty[None] < r[3][:, None])
        assert not np.any(hit & ~inside)
        ranges, ids, _ = oracle.tile_lists(m, cam.width, cam.height)
        tiles_x = (cam.width + tw - 1) // tw
        for t in range(ranges.shape[0]):
            tx0, ty0 = t % tiles_x, t // tiles_x
            want = sorted((int(m["zbits"][i]), i) for i in range(scene.n)
                          if m["valid"][i] and r[0, i] <= tx0 < r[2, i] and r[1, i] <= ty0 < r[3, i])
            assert ids[ranges[t, 0]:ranges[t, 1]].tolist() == [i for _, i in want]
