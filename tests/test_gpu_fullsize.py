"""Full-size parity for the large workloads, in the launch shape the bench
uses: per-tile lists bit-exact on sampled tiles, sampled pixels of every state
against the oracle (1e-4 plus its ambiguity budget), and the on-device PSNR
against a host PSNR of the GPU's own images."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _dev(w):
    import paper_2606_17212_amd as dgs
    dev = torch.device("cuda:0")
    return (dgs.GaussianScene.from_arrays(w.scene, dev), dgs.Camera.from_arrays(w.camera),
            torch.from_numpy(np.ascontiguousarray(w.codes)).to(dev))


def _tile_list(m, t, tiles_x):
    tx, ty = t % tiles_x, t // tiles_x
    r = m["rect"]
    sel = m["valid"] & (r[0] <= tx) & (tx < r[2]) & (r[1] <= ty) & (ty < r[3])
    ids = np.nonzero(sel)[0]
    return ids[np.lexsort((ids, m["zbits"][ids].astype(np.int64)))]


def test_full_size_2700k_1080p_256states():
    import paper_2606_17212_amd as dgs
    w = synth.make_workload("g2700k_1080p_256states", background=(0.25, 0.5, 0.75))
    scene, cam, codes = _dev(w)
    r = dgs.Renderer(tile=(16, 16), states_per_group=8)
    img = r.render(scene, cam, codes, w.basis, tuple(w.background))
    M = r.check()
    sec = r.sections(scene, cam, codes.shape[0])
    m = oracle.mirror_f32(w.scene, w.camera, w.basis)
    rect = m["rect"].astype(np.int64)
    assert M == int(np.where(m["valid"], (rect[2] - rect[0]).clip(0) * (rect[3] - rect[1]).clip(0), 0).sum())
    ranges = sec["ranges"].numpy().astype(np.int64)
    ids = sec["sorted_ids"].numpy()
    rng = np.random.default_rng(5)
    tiles = np.concatenate([rng.integers(0, ranges.shape[0], 12), np.argsort(ranges[:, 1] - ranges[:, 0])[-4:]])
    for t in tiles:
        want = _tile_list(m, int(t), sec["tiles_x"])
        assert np.array_equal(ids[ranges[t, 0]:ranges[t, 1]].astype(np.int64), want), t
    pix = np.concatenate([np.stack([rng.integers(0, 1920, 24), rng.integers(0, 1080, 24)], 1),
                          np.stack([rng.integers(760, 1160, 24), rng.integers(340, 740, 24)], 1)])
    host = img[:, pix[:, 1], pix[:, 0], :].cpu().numpy()
    ref = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background, pixels=pix)
    ex = np.abs(host.astype(np.float64) - ref["image"]).max(-1) - ref["budget"]
    assert ex.max() <= TOL, f"excess {ex.max():.3g}"
    ps = r.render(scene, cam, codes[[0, 128, 255]].contiguous(), w.basis, tuple(w.background), per_state=True)
    assert torch.equal(ps, img[[0, 128, 255]])
    # the bench's launch for this workload (groups of 16, persistent) gives the same images bit for bit
    r16 = dgs.Renderer(tile=(16, 16), states_per_group=16, persistent=True)
    assert torch.equal(r16.render(scene, cam, codes, w.basis, tuple(w.background)), img)


def test_full_size_1m_540p_psnr_batch():
    import paper_2606_17212_amd as dgs
    w = synth.make_workload("g1m_540p_32768states_psnr", background=(0.25, 0.5, 0.75))
    scene, cam, codes = _dev(w)
    bg = tuple(w.background)
    r = dgs.Renderer(tile=(16, 16), states_per_group=8)
    full = r.render(scene, cam, torch.ones_like(codes[:1]), w.basis, bg)[0].contiguous()
    img = r.render(scene, cam, codes, w.basis, bg)
    r.check()
    ps = r.render_psnr(scene, cam, codes, w.basis, full, bg).cpu().numpy().astype(np.float64)
    d = img.double() - full.double()[None]
    mse = (d * d).reshape(d.shape[0], -1).mean(1).cpu().numpy()
    host = 10 * np.log10(1 / np.maximum(mse, 1e-10))
    assert np.max(np.abs(ps - host)) <= 1e-3
    rng = np.random.default_rng(9)
    pix = np.concatenate([np.stack([rng.integers(0, 960, 24), rng.integers(0, 540, 24)], 1),
                          np.stack([rng.integers(330, 630, 24), rng.integers(120, 420, 24)], 1)])
    host_img = img[:, pix[:, 1], pix[:, 0], :].cpu().numpy()
    ref = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background, pixels=pix)
    ex = np.abs(host_img.astype(np.float64) - ref["image"]).max(-1) - ref["budget"]
    assert ex.max() <= TOL, f"excess {ex.max():.3g}"


def test_full_size_250k_800px_64states_refined():
    """The headline workload with three refinement levels, in the bench's
    launch shape: instance count from the mirrors of the four depth records,
    sampled tiles' lists (records of the Gaussian at each depth) and sampled
    pixels of every state against the per-state decode of the oracle."""
    import paper_2606_17212_amd as dgs
    w = synth.make_workload("g250k_800px_64states", background=(0.25, 0.5, 0.75))
    levels = synth.make_refinement(w.scene, index=w.index)
    dev = torch.device("cuda:0")
    scene = dgs.GaussianScene.from_arrays(w.scene, dev, refine=levels)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(np.ascontiguousarray(w.codes)).to(dev)
    r = dgs.Renderer(tile=(16, 16), states_per_group=8)
    img = r.render(scene, cam, codes, w.basis, tuple(w.background))
    M = r.check()
    sec = r.sections(scene, cam, codes.shape[0])
    n = w.scene.n
    layer = (w.scene.packet_layer & 3).astype(np.int64)
    # record 4 i + d: Gaussian i at depth d, present when layer_i <= d
    zb = np.zeros(4 * n, np.uint32)
    rect = np.zeros((4, 4 * n), np.int64)
    valid = np.zeros(4 * n, bool)
    for d in range(4):
        m = oracle.mirror_f32(oracle.refined_scene(w.scene, levels, np.full(w.scene.num_packets, d + 1, np.uint8)),
                              w.camera, w.basis)
        zb[d::4] = m["zbits"]
        rect[:, d::4] = m["rect"]
        valid[d::4] = m["valid"] & (layer <= d)
    mm = dict(zbits=zb, rect=rect, valid=valid)
    assert M == int(np.where(valid, (rect[2] - rect[0]).clip(0) * (rect[3] - rect[1]).clip(0), 0).sum())
    ranges = sec["ranges"].numpy().astype(np.int64)
    ids = sec["sorted_ids"].numpy()
    rng = np.random.default_rng(6)
    tiles = np.concatenate([rng.integers(0, ranges.shape[0], 8), np.argsort(ranges[:, 1] - ranges[:, 0])[-3:]])
    for t in tiles:
        want = _tile_list(mm, int(t), sec["tiles_x"])
        assert np.array_equal(ids[ranges[t, 0]:ranges[t, 1]].astype(np.int64), want), t
    pix = np.concatenate([np.stack([rng.integers(0, 800, 12), rng.integers(0, 800, 12)], 1),
                          np.stack([rng.integers(250, 550, 12), rng.integers(250, 550, 12)], 1)])
    host = img[:, pix[:, 1], pix[:, 0], :].cpu().numpy()
    ref = oracle.render_refined(w.scene, levels, w.camera, w.basis, w.codes, w.background, pixels=pix)
    ex = np.abs(host.astype(np.float64) - ref["image"]).max(-1) - ref["budget"]
    assert ex.max() <= TOL, f"excess {ex.max():.3g}"


def test_full_size_utility_1m_540p_64groups_16contexts():
    """Eq. (3) at the utility bench's size and launch shape: every delta of
    the paired incremental renderer equals the difference of the on-device
    distortions of full-frame renders of both states (whose images the
    parity tests pin to the oracle), and Eq. (4) of the device deltas equals
    the oracle's risk adjustment of the same values."""
    import paper_2606_17212_amd as dgs
    from oracle import utility as U
    uw = synth.make_utility_workload("g1m_540p_utility_64groups_16contexts")
    w = uw.base
    dev = torch.device("cuda:0")
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    bg = tuple(float(x) for x in w.background)
    ctx = torch.from_numpy(uw.codes).to(dev)
    cg = torch.from_numpy(uw.context_group).to(dev)
    gpl = torch.from_numpy(uw.group_pl.view(np.int16)).to(dev)
    G, J = int(gpl.shape[0]), int(ctx.shape[0])
    r = dgs.Renderer(dev, tile=(16, 16), states_per_group=8)
    r.plan(scene, cam, w.basis, 512)
    ref = r.render(scene, cam, torch.full_like(ctx[:1], 4), w.basis, bg)[0].contiguous()
    r.bin(scene, cam, w.basis)
    delta = r.utility(scene, cam, ctx, cg, gpl, w.basis, ref, bg)
    assert r.utility_check() > 0
    mg = uw.codes.copy()
    p = (uw.group_pl >> 2).astype(np.int64)[uw.context_group]
    mg[np.arange(J), p] = (uw.group_pl & 3).astype(np.uint8)[uw.context_group] + 1
    mg = torch.from_numpy(mg).to(dev)
    full = np.zeros(J)
    for b in range(0, J, 256):
        e = min(J, b + 256)
        imgs = r.render(scene, cam, torch.cat([ctx[b:e], mg[b:e]]).contiguous(), w.basis, bg)
        d = dgs.distortion(imgs, ref).double().cpu().numpy()
        full[b:e] = d[:e - b] - d[e - b:]
    dl = delta.double().cpu().numpy()
    assert np.abs(dl - full).max() <= 1e-6, np.abs(dl - full).max()
    assert np.abs(full).max() > 1e-5
    offsets = np.searchsorted(uw.context_group, np.arange(G + 1)).astype(np.int32)
    stats = dgs.risk_adjusted(delta, torch.from_numpy(offsets).to(dev)).cpu().numpy().astype(np.float64)
    vals = delta.cpu().numpy().astype(np.float64)
    for g in range(G):
        want = U.risk_adjusted(vals[offsets[g]:offsets[g + 1]])
        got = stats[g]
        assert np.allclose(got, [want["mean"], want["quantile"], want["std"], want["risk_adjusted"]],
                           rtol=1e-5, atol=1e-9), (g, got, want)
