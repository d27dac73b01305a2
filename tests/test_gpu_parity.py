"""GPU parity: the HIP path through the C ABI against the oracle.

Bars: tile rectangles, depth keys and per-tile sorted lists bit-exact with the
oracle's FP32 mirror; images within 1e-4 absolute of the FP64 oracle plus its
ambiguity budget (pairs whose FP32 exponent or transmittance may fall on the
other side of the 1/255 skip or the 1e-4 stop, from the mirror's FP32 records;
the premises of that bound -- records bit-exact with the mirror, log2-opacity
within 2^-16 -- are checked here too);
batched == per-state == any group size == either tile shape, bit for bit.
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
BG = (0.25, 0.5, 0.75)
TOL = 1e-4


def _dgs():
    import paper_2606_17212_amd as dgs
    return dgs


def on_device(w):
    dgs = _dgs()
    dev = torch.device("cuda:0")
    return (dgs.GaussianScene.from_arrays(w.scene, dev), dgs.Camera.from_arrays(w.camera),
            torch.from_numpy(np.ascontiguousarray(w.codes)).to(dev))


def image_excess(gpu_img, ref):
    """max over pixels of (|gpu - oracle| - budget), per state/pixel/channel."""
    d = np.abs(gpu_img.astype(np.float64) - ref["image"]).max(-1)
    return d - ref["budget"]


@pytest.fixture(scope="module")
def tiny():
    w = synth.make_workload("g4k_128px_16states", background=BG)
    ref = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background)
    return w, ref


@pytest.mark.parametrize("tile", [(16, 16), (32, 8)])
def test_geometry_keys_rects_and_lists_bit_exact(tiny, tile):
    dgs = _dgs()
    w, _ = tiny
    scene, cam, codes = on_device(w)
    r = dgs.Renderer(tile=tile)
    r.render(scene, cam, codes, w.basis, BG)
    assert r.check() > 0
    sec = r.sections(scene, cam, codes.shape[0])
    m = oracle.mirror_f32(w.scene, w.camera, w.basis, *tile)
    valid = m["valid"]
    zb = sec["rec1"][:, 3].numpy().view(np.uint32)
    assert np.array_equal(zb[valid], m["zbits"][valid])
    rect = sec["rect"].numpy().view(np.uint32)
    x0, y0 = rect[:, 0] & 0xFFFF, rect[:, 0] >> 16
    x1, y1 = rect[:, 1] & 0xFFFF, rect[:, 1] >> 16
    gr = np.stack([x0, y0, x1, y1]).astype(np.int64)
    assert np.array_equal(gr[:, valid], m["rect"][:, valid].astype(np.int64))
    ranges, ids, _ = oracle.tile_lists(m, w.camera.width, w.camera.height)
    granges = sec["ranges"].numpy().astype(np.int64)
    nonempty = ranges[:, 1] > ranges[:, 0]
    assert np.array_equal(granges[nonempty], ranges[nonempty])
    assert np.all(granges[~nonempty, 1] == granges[~nonempty, 0])
    M = ids.size
    assert np.array_equal(sec["sorted_ids"].numpy()[:M].astype(np.int64), ids)
    # FP32 projection against the FP64 definition
    g = oracle.geometry_f64(w.scene, w.camera, w.basis)
    # wave-block reach masks are conservative: a tile's 8x8 block holding a
    # pixel centre where the Gaussian's FP64 alpha >= 1/255 has its bit set
    masks = sec["wave_masks"].numpy()[:M].astype(np.int64)
    tile_of = np.repeat(np.arange(ranges.shape[0]), ranges[:, 1] - ranges[:, 0])
    tiles_x = sec["tiles_x"]
    need_any = np.zeros((M, 4), bool)
    for b in range(4):
        bx, by = (8 * b) % tile[0], ((8 * b) // tile[0]) * 8
        px = (tile_of % tiles_x) * tile[0] + bx
        py = (tile_of // tiles_x) * tile[1] + by
        for dy in range(8):
            for dx in range(8):
                x = px + dx + 0.5 - g["u"][ids]
                y = py + dy + 0.5 - g["v"][ids]
                q = g["conA"][ids] * x * x + 2 * g["conB"][ids] * x * y + g["conC"][ids] * y * y
                inside = (px + dx < w.camera.width) & (py + dy < w.camera.height)
                need_any[:, b] |= inside & (g["o"][ids] * np.exp(-0.5 * q) >= 1 / 255)
    bits = (masks[:, None] >> np.arange(4)[None, :]) & 1
    assert not np.any(need_any & (bits == 0)), "a reached wave block has no mask bit"
    assert bits.sum() < 4 * M  # and the masks do cull blocks
    # premises of the oracle's ambiguity budget: the compositing records hold
    # the mirror's FP32 (u, v) and scaled conic bit for bit, and a log2-opacity
    # within 2^-16 of the FP64 value
    r0, r1 = sec["rec0"].numpy(), sec["rec1"].numpy()
    assert np.array_equal(r0[valid, 0].view(np.uint32), m["u"][valid].view(np.uint32))
    assert np.array_equal(r0[valid, 1].view(np.uint32), m["v"][valid].view(np.uint32))
    for j, k in enumerate(("cA", "cB", "cC")):
        assert np.array_equal(r1[valid, j].view(np.uint32), m[k][valid].view(np.uint32)), k
    assert np.max(np.abs(r0[valid, 2].astype(np.float64) - np.log2(g["o"][valid]))) <= 2.0 ** -16
    rec0, rec1, rec2 = (sec[k].numpy().astype(np.float64) for k in ("rec0", "rec1", "rec2"))
    assert np.max(np.abs(rec0[valid, 0] - g["u"][valid])) < 2e-4
    assert np.max(np.abs(rec0[valid, 1] - g["v"][valid])) < 2e-4
    # records hold log2(opacity) and the conic scaled by (-log2(e)/2, -log2(e), -log2(e)/2)
    assert np.max(np.abs(np.exp2(rec0[valid, 2]) / g["o"][valid] - 1)) < 1e-5
    l2e = 1.0 / np.log(2.0)
    conic = np.stack([rec1[:, 0] / (-0.5 * l2e), rec1[:, 1] / (-l2e), rec1[:, 2] / (-0.5 * l2e)], 1)
    for j, k in enumerate(("conA", "conB", "conC")):
        scale = np.maximum(np.abs(g["conA"]), np.abs(g["conC"]))[valid]
        assert np.max(np.abs(conic[valid, j] - g[k][valid]) / scale) < 2e-5
    col = np.stack([g["r"], g["g"], g["b_"]], 1)[valid]
    assert np.max(np.abs(rec2[valid, :3] - col)) < 2e-6


@pytest.mark.parametrize("tile,S", [((16, 16), 16), ((32, 8), 4), ((16, 16), 1)])
def test_images_match_oracle(tiny, tile, S):
    dgs = _dgs()
    w, ref = tiny
    scene, cam, codes = on_device(w)
    r = dgs.Renderer(tile=tile, states_per_group=S)
    img, tf = r.render(scene, cam, codes, w.basis, BG, tfinal=True)
    r.check()
    ex = image_excess(img.cpu().numpy(), ref)
    assert ex.max() <= TOL, f"max excess {ex.max():.3g} at {np.unravel_index(ex.argmax(), ex.shape)}"
    tfe = np.abs(tf.cpu().numpy() - ref["tfinal"])
    amb = ref["budget"] > 0
    assert tfe[~amb].max() <= 1e-5


def test_batched_equals_per_state_and_any_launch_shape(tiny):
    dgs = _dgs()
    w, _ = tiny
    scene, cam, codes = on_device(w)
    base = dgs.Renderer(tile=(16, 16), states_per_group=16)
    ref_img, ref_tf = base.render(scene, cam, codes, w.basis, BG, tfinal=True)
    ps_img, ps_tf = base.render(scene, cam, codes, w.basis, BG, tfinal=True, per_state=True)
    base.check()
    assert torch.equal(ps_img, ref_img) and torch.equal(ps_tf, ref_tf)
    for tile in ((16, 16), (32, 8)):
        for S in (1, 2, 4, 8, 16, 32):
            r = dgs.Renderer(tile=tile, states_per_group=S)
            img = r.render(scene, cam, codes, w.basis, BG)
            assert torch.equal(img, ref_img), (tile, S)
    # repeat-run determinism
    assert torch.equal(base.render(scene, cam, codes, w.basis, BG), ref_img)


def test_persistent_launch_equals_grid_launch(tiny):
    """The persistent launch (workgroups draining per-XCD queues) computes
    every (tile, state group) item exactly as the grid launch does: images,
    final transmittances and PSNR bit-identical, also on a second call that
    reuses the queues with fewer states."""
    dgs = _dgs()
    w, _ = tiny
    scene, cam, codes = on_device(w)
    for tile in ((16, 16), (32, 8)):
        for S in (1, 8, 32):
            g = dgs.Renderer(tile=tile, states_per_group=S)
            p = dgs.Renderer(tile=tile, states_per_group=S, persistent=True)
            for c in (codes, codes[: max(1, codes.shape[0] // 3)].contiguous()):
                gi, gt = g.render(scene, cam, c, w.basis, BG, tfinal=True)
                pi, pt = p.render(scene, cam, c, w.basis, BG, tfinal=True)
                assert torch.equal(pi, gi) and torch.equal(pt, gt), (tile, S, c.shape[0])
                ref = gi[0].contiguous()
                assert torch.equal(p.render_psnr(scene, cam, c, w.basis, ref, BG),
                                   g.render_psnr(scene, cam, c, w.basis, ref, BG))
            p.check()
            assert p.composite_stats(scene, cam, codes, w.basis) == g.composite_stats(scene, cam, codes, w.basis)


def test_state_permutation_and_masks(tiny):
    dgs = _dgs()
    w, _ = tiny
    scene, cam, codes = on_device(w)
    r = dgs.Renderer()
    img = r.render(scene, cam, codes, w.basis, BG)
    perm = torch.randperm(codes.shape[0], generator=torch.Generator().manual_seed(0)).to(codes.device)
    img_p = r.render(scene, cam, codes[perm].contiguous(), w.basis, BG)
    assert torch.equal(img_p, img[perm])
    empty = torch.zeros_like(codes[:3])
    e = r.render(scene, cam, empty, w.basis, BG)
    assert torch.equal(e, torch.tensor(BG, dtype=torch.float32, device=e.device).expand_as(e))
    full = torch.full_like(codes[:2], 4)
    one = torch.ones_like(codes[:2])  # this scene has only layer 0: code 1 delivers everything
    assert torch.equal(r.render(scene, cam, full, w.basis, BG), r.render(scene, cam, one, w.basis, BG))


def test_storage_permutation_invariance(tiny):
    dgs = _dgs()
    w, _ = tiny
    m = oracle.mirror_f32(w.scene, w.camera, w.basis)
    # random storage order, except that Gaussians with equal depth keys keep
    # their relative order (equal keys are ordered by storage index)
    perm = np.random.default_rng(4).permutation(w.scene.n)
    newpos = np.empty_like(perm)
    newpos[perm] = np.arange(perm.size)
    zb = m["zbits"]
    _, inv, cnt = np.unique(zb, return_inverse=True, return_counts=True)
    for grp in np.nonzero(cnt > 1)[0]:
        members = np.nonzero(inv == grp)[0]
        newpos[members] = np.sort(newpos[members])
    perm = np.empty_like(newpos)
    perm[newpos] = np.arange(newpos.size)
    scene, cam, codes = on_device(w)
    w2 = synth.Workload(**{**w.__dict__, "scene": synth.permute_gaussians(w.scene, perm)})
    scene2, _, _ = on_device(w2)
    r = dgs.Renderer()
    a = r.render(scene, cam, codes, w.basis, BG)
    b = r.render(scene2, cam, codes, w.basis, BG)
    assert torch.equal(a, b)


def test_ragged_sizes_and_edge_cases():
    dgs = _dgs()
    sc = synth.make_scene(1537, 4, 4, 4, "sh1", index=9)
    cam = synth.ring_camera(100, 75)
    codes = synth.make_codes("present_depth", 0.3, 1.0, 5, sc.num_packets, 4, index=9)
    w = synth.Workload("ragged", 9, sc, cam, codes, synth.temporal_basis(0.5, 2), 0.5,
                       np.array(BG, np.float32))
    ref = oracle.render(sc, cam, w.basis, codes, w.background)
    scene, dcam, dcodes = on_device(w)
    for tile in ((16, 16), (32, 8)):
        r = dgs.Renderer(tile=tile, states_per_group=4)
        img = r.render(scene, dcam, dcodes, w.basis, BG)
        r.check()
        assert image_excess(img.cpu().numpy(), ref).max() <= TOL
        ps = r.render(scene, dcam, dcodes, w.basis, BG, per_state=True)
        assert torch.equal(ps, img)
    # no states: nothing to do; one state
    r = dgs.Renderer()
    one = r.render(scene, dcam, dcodes[:1].contiguous(), w.basis, BG)
    assert one.shape == (1, 75, 100, 3)
    assert image_excess(one.cpu().numpy(), {k: v[:1] for k, v in ref.items()}).max() <= TOL


def test_camera_inside_and_behind():
    """Gaussians behind the camera and on the near plane are culled; the
    camera sits inside the cloud."""
    dgs = _dgs()
    sc = synth.make_scene(3000, 4, 2, 1, "rgb", index=10)
    cam = synth.ring_camera(96, 64, radius=0.5)
    codes = synth.make_codes("bernoulli", 0.8, 0.8, 3, sc.num_packets, 1, index=10)
    w = synth.Workload("inside", 10, sc, cam, codes, synth.temporal_basis(0.5, 2), 0.5,
                       np.array(BG, np.float32))
    ref = oracle.render(sc, cam, w.basis, codes, w.background)
    scene, dcam, dcodes = on_device(w)
    r = dgs.Renderer()
    img = r.render(scene, dcam, dcodes, w.basis, BG)
    r.check()
    assert image_excess(img.cpu().numpy(), ref).max() <= TOL


def test_overflow_is_reported_and_safe(tiny):
    dgs = _dgs()
    w, _ = tiny
    scene, cam, codes = on_device(w)
    r = dgs.Renderer()
    r.plan(scene, cam, w.basis, codes.shape[0])
    r.capacity = 100  # far below the scene's instances; the workspace stays large enough
    img = r.render(scene, cam, codes, w.basis, BG)
    with pytest.raises(dgs.DgsError) as e:
        r.check()
    assert e.value.status == 3
    assert torch.equal(img, torch.tensor(BG, dtype=torch.float32, device=img.device).expand_as(img))


def test_psnr_reduction(tiny):
    dgs = _dgs()
    w, ref = tiny
    scene, cam, codes = on_device(w)
    r = dgs.Renderer()
    full = torch.ones_like(codes[:1])
    reference = r.render(scene, cam, full, w.basis, BG)[0].contiguous()
    img = r.render(scene, cam, codes, w.basis, BG)
    ps = r.render_psnr(scene, cam, codes, w.basis, reference, BG).cpu().numpy()
    host = oracle.psnr(img.cpu().numpy(), reference.cpu().numpy())
    assert np.max(np.abs(ps - host)) <= 1e-4 * np.maximum(1.0, np.abs(host)).max()
    ref_full = oracle.render(w.scene, w.camera, w.basis, np.ones_like(w.codes[:1]), w.background)
    orc = oracle.psnr(ref["image"], ref_full["image"][0])
    assert np.max(np.abs(ps - orc)) <= 0.05


def test_full_size_250k_800px_sampled_pixels():
    """The 250k-Gaussian, 800x800, 64-state workload in the bench's launch
    shape: sorted lists bit-exact at full size, sampled pixels of every state
    against the oracle, and per-state == batched for a few states."""
    dgs = _dgs()
    w = synth.make_workload("g250k_800px_64states", background=BG)
    scene, cam, codes = on_device(w)
    r = dgs.Renderer(tile=(16, 16), states_per_group=16)
    img = r.render(scene, cam, codes, w.basis, BG)
    M = r.check()
    sec = r.sections(scene, cam, codes.shape[0])
    m = oracle.mirror_f32(w.scene, w.camera, w.basis)
    ranges, ids, _ = oracle.tile_lists(m, w.camera.width, w.camera.height)
    assert M == ids.size
    assert np.array_equal(sec["sorted_ids"].numpy()[:M].astype(np.int64), ids)
    rng = np.random.default_rng(12)
    pix = np.concatenate([rng.integers(0, 800, size=(96, 2)),
                          rng.integers(300, 500, size=(96, 2))])  # more in the dense centre
    ref = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background, pixels=pix)
    got = img.cpu().numpy()[:, pix[:, 1], pix[:, 0], :]
    ex = np.abs(got.astype(np.float64) - ref["image"]).max(-1) - ref["budget"]
    assert ex.max() <= TOL, f"excess {ex.max():.3g}"
    sub = codes[[0, 17, 63]].contiguous()
    ps = r.render(scene, cam, sub, w.basis, BG, per_state=True)
    assert torch.equal(ps, img[[0, 17, 63]])


def test_full_size_250k_800px_lists_and_masks_32x8():
    """The same workload binned with 32x8 tiles (the level-2 scatter's other
    tile width): tile ranges and sorted lists bit-exact at full size, and on a
    sample of the instances every 8x8 block holding a pixel centre where the
    Gaussian's FP64 alpha reaches 1/255 has its mask bit."""
    dgs = _dgs()
    w = synth.make_workload("g250k_800px_64states", background=BG)
    scene, cam, codes = on_device(w)
    r = dgs.Renderer(tile=(32, 8), states_per_group=8)
    r.render(scene, cam, codes, w.basis, BG)
    M = r.check()
    sec = r.sections(scene, cam, codes.shape[0])
    m = oracle.mirror_f32(w.scene, w.camera, w.basis, 32, 8)
    ranges, ids, _ = oracle.tile_lists(m, w.camera.width, w.camera.height)
    assert M == ids.size
    granges = sec["ranges"].numpy().astype(np.int64)
    nonempty = ranges[:, 1] > ranges[:, 0]
    assert np.array_equal(granges[nonempty], ranges[nonempty])
    assert np.array_equal(sec["sorted_ids"].numpy()[:M].astype(np.int64), ids)
    g = oracle.geometry_f64(w.scene, w.camera, w.basis)
    rng = np.random.default_rng(5)
    pick = rng.choice(M, size=20000, replace=False)
    sid = ids[pick]
    masks = sec["wave_masks"].numpy()[:M].astype(np.int64)[pick]
    tile_of = np.repeat(np.arange(ranges.shape[0]), ranges[:, 1] - ranges[:, 0])[pick]
    tiles_x = sec["tiles_x"]
    need = np.zeros((pick.size, 4), bool)
    for b in range(4):  # 32x8 tiles: four 8x8 blocks side by side
        px = (tile_of % tiles_x) * 32 + 8 * b
        py = (tile_of // tiles_x) * 8
        for dy in range(8):
            for dx in range(8):
                x = px + dx + 0.5 - g["u"][sid]
                y = py + dy + 0.5 - g["v"][sid]
                q = g["conA"][sid] * x * x + 2 * g["conB"][sid] * x * y + g["conC"][sid] * y * y
                inside = (px + dx < w.camera.width) & (py + dy < w.camera.height)
                need[:, b] |= inside & (g["o"][sid] * np.exp(-0.5 * q) >= 1 / 255)
    bits = (masks[:, None] >> np.arange(4)[None, :]) & 1
    assert not np.any(need & (bits == 0)), "a reached wave block has no mask bit"
    assert bits.sum() < 4 * pick.size


def test_bin_once_composite_many_and_work_counters(tiny):
    """One binning serves several composite calls (a sweep over state
    batches); the blend counter equals the oracle's composited-pair count up to
    ambiguous pixels."""
    dgs = _dgs()
    w, ref = tiny
    scene, cam, codes = on_device(w)
    r = dgs.Renderer(states_per_group=8)
    full = r.render(scene, cam, codes, w.basis, BG)
    r.bin(scene, cam, w.basis)
    a = r.composite(scene, cam, codes[:5].contiguous(), w.basis, BG)
    b = r.composite(scene, cam, codes[5:].contiguous(), w.basis, BG)
    assert torch.equal(torch.cat([a, b]), full)
    alpha_evals, blends, wave_evals, wave_miss = r.composite_stats(scene, cam, codes, w.basis)
    assert 0 <= wave_miss <= wave_evals and wave_evals * 64 >= alpha_evals
    want = int(ref["ncomp"].sum())
    amb = int((ref["budget"] > 0).sum())
    assert abs(blends - want) <= 4 * amb, (blends, want, amb)
    assert alpha_evals >= blends / codes.shape[0]
    ps = r.composite_psnr(scene, cam, codes, w.basis, full[0].contiguous(), BG).cpu().numpy()
    host = oracle.psnr(full.cpu().numpy(), full[0].cpu().numpy())
    assert np.max(np.abs(ps - host)) <= 1e-3


def test_lds_batch_sizes_give_identical_results():
    """Staging 128, 256 or 512 list entries per LDS batch changes the batch
    boundaries only: with tile lists of ~500 to ~5700 entries (ragged against
    every batch size), images and final transmittances are bit-identical for
    every tile shape, group size and launch, and match the oracle; PSNR is
    bit-identical for a given tile shape.  Groups
    of fewer than 4 states run the 256-entry variant whatever is asked."""
    dgs = _dgs()
    w = synth.subscene(12000, 96, 80, states=12, log_scale_mean=-2.2, index=9, background=BG)
    ref = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background)
    scene, cam, codes = on_device(w)
    base = dgs.Renderer(tile=(16, 16), states_per_group=8)
    bi, bt = base.render(scene, cam, codes, w.basis, BG, tfinal=True)
    base.check()
    ex = image_excess(bi.cpu().numpy(), ref)
    assert ex.max() <= TOL, ex.max()
    rng = base.sections(scene, cam, codes.shape[0])["ranges"].numpy().astype(np.int64)
    lens = rng[:, 1] - rng[:, 0]
    assert lens.max() > 4 * 512 and np.any(lens % 512 != 0) and np.any(lens % 128 != 0)
    target = bi[0].contiguous()
    for tile in ((16, 16), (32, 8)):
        # PSNR sums per-tile partials, so its last bits depend on the tile shape only
        bp = dgs.Renderer(tile=tile, states_per_group=8).render_psnr(scene, cam, codes, w.basis, target, BG)
        for S in (4, 8, 32):
            for pers in (False, True):
                for B in (128, 512, 256):
                    r = dgs.Renderer(tile=tile, states_per_group=S, persistent=pers, lds_batch=B)
                    assert r.launch_plan(cam, codes.shape[0])["lds_batch"] == B
                    img, tf = r.render(scene, cam, codes, w.basis, BG, tfinal=True)
                    assert torch.equal(img, bi) and torch.equal(tf, bt), (tile, S, pers, B)
                    assert torch.equal(r.render_psnr(scene, cam, codes, w.basis, target, BG), bp), (tile, S, pers, B)
                    r.check()
    for S in (1, 2):
        r = dgs.Renderer(states_per_group=S, lds_batch=512)
        assert r.launch_plan(cam, codes.shape[0])["lds_batch"] == 256
        assert torch.equal(r.render(scene, cam, codes, w.basis, BG), bi), S
    with pytest.raises(ValueError, match="lds_batch"):
        dgs.Renderer(lds_batch=64).render(scene, cam, codes, w.basis, BG)
