"""Counterfactual render utility on the GPU (Eq. (3)-(4), D of Sec. 4):
distortion and risk adjustment against the oracle, the paired incremental
renderer against the oracle's full renders and against the GPU's own
full-frame path, and its error handling."""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import utility as U

pytestmark = pytest.mark.gpu
BG = (0.25, 0.5, 0.75)


def _dgs():
    import paper_2606_17212_amd as dgs
    return dgs


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).to("cuda:0")


@pytest.mark.parametrize("shape", [(3, 37, 53), (2, 16, 16), (1, 7, 5), (2, 80, 96)])
def test_distortion_matches_oracle(shape):
    dgs = _dgs()
    W, H, Wd = shape
    rng = np.random.default_rng(11 + H)
    ref = rng.uniform(0, 1, (H, Wd, 3)).astype(np.float32)
    imgs = np.clip(ref[None] + rng.normal(0, 0.05, (W, H, Wd, 3)), 0, 1.2).astype(np.float32)
    imgs[0, : H // 2] = 0.3  # a flat region (sigma = 0 windows)
    d = dgs.distortion(_dev(imgs), _dev(ref)).cpu().numpy()
    want = np.array([U.distortion(imgs[k], ref) for k in range(W)])
    # FP32 window moments of shifted values: per-pixel SSIM error <~ 1e-6,
    # averaged over the image
    assert np.abs(d - want).max() <= 2e-6, (d, want)
    assert abs(dgs.distortion(_dev(ref[None]), _dev(ref)).item()) <= 1e-6


def test_risk_adjusted_matches_oracle():
    dgs = _dgs()
    rng = np.random.default_rng(12)
    counts = [1, 2, 7, 100, 1000, 4096]
    vals = [rng.normal(0.001, 0.002, c) for c in counts]
    flat = np.concatenate(vals).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    out = dgs.risk_adjusted(_dev(flat), _dev(off)).cpu().numpy().astype(np.float64)
    for k, v in enumerate(vals):
        r = U.risk_adjusted(v.astype(np.float32).astype(np.float64))
        want = np.array([r["mean"], r["quantile"], r["std"], r["risk_adjusted"]])
        assert np.allclose(out[k], want, rtol=1e-5, atol=1e-9), (k, out[k], want)
    # a NaN value or an out-of-range count makes the group's four outputs NaN
    flat2 = np.array([1, np.nan, 3, 4, 5], np.float32)
    off2 = np.array([0, 2, 2, 5], np.int32)
    o2 = dgs.risk_adjusted(_dev(flat2), _dev(off2)).cpu().numpy()
    assert np.all(np.isnan(o2[0])) and np.all(np.isnan(o2[1])) and np.allclose(o2[2], [4, 3.2, np.sqrt(2 / 3), o2[2, 3]])


def _utility_case(n=3000, seed=7, J_per=3):
    """16 packets x 4 layers, 96x80 (ragged tiles); groups (packet, layer)
    with contexts holding the packet at exactly that depth."""
    scene = synth.make_scene(n, 4, 4, 4, "sh1", index=7, stream=0)
    scene.log_scale[:] += np.float32(0.4)
    cam = synth.ring_camera(96, 80)
    basis = synth.temporal_basis(0.5, scene.rank)
    rng = np.random.default_rng(seed)
    groups = [(0, 0), (3, 1), (5, 2), (9, 3), (14, 0), (6, 1)]
    P = scene.num_packets
    ctx, cg = [], []
    for k, (p, l) in enumerate(groups):
        c = rng.integers(0, 5, (J_per, P)).astype(np.uint8)
        c[:, p] = l
        ctx.append(c)
        cg += [k] * J_per
    ctx = np.concatenate(ctx)
    full = np.full((1, P), 4, np.uint8)
    ref = oracle.render(scene, cam, basis, full, np.asarray(BG))["image"][0].astype(np.float32)
    return scene, cam, basis, groups, ctx, np.asarray(cg, np.int32), ref


def test_utility_matches_oracle_and_full_frame_path():
    dgs = _dgs()
    scene, cam, basis, groups, ctx, cg, ref = _utility_case()
    dev = torch.device("cuda:0")
    s = dgs.GaussianScene.from_arrays(scene, dev)
    c = dgs.Camera.from_arrays(cam)
    gpl = np.array([(p << 2) | l for p, l in groups], np.uint16).view(np.int16)
    for tile in ((16, 16), (32, 8)):
        r = dgs.Renderer(dev, tile=tile, states_per_group=8)
        r.plan(s, c, basis, 1)
        r.bin(s, c, basis)
        delta = r.utility(s, c, _dev(ctx), _dev(cg), _dev(gpl), basis, _dev(ref), BG).cpu().numpy()
        assert r.utility_check() > 0
        # the GPU's own full-frame path: render m and m u g, D of each
        mg = ctx.copy()
        for j in range(len(ctx)):
            p, l = groups[cg[j]]
            mg[j, p] = l + 1
        both = r.render(s, c, _dev(np.concatenate([ctx, mg])), basis, BG)
        d = dgs.distortion(both, _dev(ref)).double().cpu().numpy()
        full = d[: len(ctx)] - d[len(ctx):]
        assert np.abs(delta - full).max() <= 1e-6, (tile, np.abs(delta - full).max())
        # the oracle: FP64 full renders of both states of every pair
        want = np.concatenate([U.deltas(scene, cam, basis, ctx[cg == k], p, l, ref, np.asarray(BG))
                               for k, (p, l) in enumerate(groups)])
        err = np.abs(delta.astype(np.float64) - want)
        assert err.max() <= 1e-5 + 1e-3 * np.abs(want).max(), (tile, err.max(), np.abs(want).max())
        assert np.abs(want).max() > 1e-4  # the groups change the image


def test_utility_edge_cases_and_errors():
    dgs = _dgs()
    scene, cam, basis, groups, ctx, cg, ref = _utility_case(n=800, J_per=2)
    dev = torch.device("cuda:0")
    s = dgs.GaussianScene.from_arrays(scene, dev)
    c = dgs.Camera.from_arrays(cam)
    gpl = np.array([(p << 2) | l for p, l in groups], np.uint16).view(np.int16)
    r = dgs.Renderer(dev)
    r.plan(s, c, basis, 1)
    r.bin(s, c, basis)
    n_items = r.utility_items(s, c, _dev(ctx), _dev(cg), _dev(gpl), basis)
    ok = r.utility(s, c, _dev(ctx), _dev(cg), _dev(gpl), basis, _dev(ref), BG, item_capacity=n_items)
    assert r.utility_check() == n_items and torch.isfinite(ok).all()
    # no contexts
    empty = r.utility(s, c, _dev(ctx[:0]), _dev(cg[:0]), _dev(gpl), basis, _dev(ref), BG, item_capacity=0)
    assert empty.numel() == 0
    # a capacity below the items needed: every delta NaN, overflow reported, nothing written out of bounds
    small = r.utility(s, c, _dev(ctx), _dev(cg), _dev(gpl), basis, _dev(ref), BG, item_capacity=max(n_items // 3, 1))
    assert torch.isnan(small).all()
    with pytest.raises(dgs.DgsError) as e:
        r.utility_check()
    assert e.value.status == 3
    # a context lacking its group's packet at the group's layer -> NaN for it, error reported
    bad = ctx.copy()
    p0, l0 = groups[cg[0]]
    bad[0, p0] = l0 + 1
    d = r.utility(s, c, _dev(bad), _dev(cg), _dev(gpl), basis, _dev(ref), BG, item_capacity=n_items)
    with pytest.raises(dgs.DgsError) as e:
        r.utility_check()
    assert e.value.status == 1
    d = d.cpu().numpy()
    assert np.isnan(d[0]) and np.allclose(d[1:], ok.cpu().numpy()[1:], rtol=0, atol=0)
    # two groups naming one (packet, layer)
    dup = np.concatenate([gpl, gpl[:1]])
    with pytest.raises(dgs.DgsError):
        r.utility_items(s, c, _dev(ctx), _dev(cg), _dev(dup), basis)
    # a group whose Gaussians are all outside the view: Delta = 0 exactly
    far = synth.make_scene(64, 1, 1, 1, "sh1", index=9, stream=0)
    far.mean[2, :] = -10.0  # behind the camera
    sf = dgs.GaussianScene.from_arrays(far, dev)
    r2 = dgs.Renderer(dev)
    r2.plan(sf, c, basis, 1)
    r2.bin(sf, c, basis)
    z = r2.utility(sf, c, _dev(np.zeros((2, 1), np.uint8)), _dev(np.zeros(2, np.int32)),
                   _dev(np.zeros(1, np.int16)), basis, _dev(ref), BG)
    assert r2.utility_check() == 0 and torch.equal(z, torch.zeros_like(z))


def test_utility_bundles_do_not_change_deltas():
    """Contexts of one group are composited four at a time; the deltas are
    the same bit for bit whatever the context order (runs of one group, mixed
    groups, a bad context in the middle)."""
    dgs = _dgs()
    scene, cam, basis, groups, ctx, cg, ref = _utility_case(n=2000, J_per=8)
    dev = torch.device("cuda:0")
    s = dgs.GaussianScene.from_arrays(scene, dev)
    c = dgs.Camera.from_arrays(cam)
    gpl = np.array([(p << 2) | l for p, l in groups], np.uint16).view(np.int16)
    r = dgs.Renderer(dev)
    r.plan(s, c, basis, 1)
    r.bin(s, c, basis)
    base = r.utility(s, c, _dev(ctx), _dev(cg), _dev(gpl), basis, _dev(ref), BG).cpu().numpy()
    n_items = r.utility_check()
    assert n_items > 0 and np.isfinite(base).all()
    rng = np.random.default_rng(3)
    for _ in range(2):
        perm = rng.permutation(len(ctx))
        d = r.utility(s, c, _dev(ctx[perm]), _dev(cg[perm]), _dev(gpl), basis, _dev(ref), BG).cpu().numpy()
        r.utility_check()
        assert np.array_equal(d, base[perm])
    # a context without its group's packet at the group's layer inside a run
    bad = ctx.copy()
    p0, l0 = groups[cg[5]]
    bad[5, p0] = l0 + 1
    d = r.utility(s, c, _dev(bad), _dev(cg), _dev(gpl), basis, _dev(ref), BG, item_capacity=n_items)
    with pytest.raises(dgs.DgsError):
        r.utility_check()
    d = d.cpu().numpy()
    assert np.isnan(d[5]) and np.array_equal(np.delete(d, 5), np.delete(base, 5))


def test_utility_with_refinement_levels():
    """Scenes with refinement levels: adding group (p, l) moves packet p from
    depth l - 1 to depth l; the paired renderer against the oracle's refined
    renders and against the GPU's own refined full-frame path."""
    dgs = _dgs()
    scene, cam, basis, groups, ctx, cg, _ = _utility_case(J_per=3)
    levels = synth.make_refinement(scene, index=7)
    P = scene.num_packets
    ref = oracle.render_refined(scene, levels, cam, basis, np.full((1, P), 4, np.uint8),
                                np.asarray(BG))["image"][0].astype(np.float32)
    dev = torch.device("cuda:0")
    s = dgs.GaussianScene.from_arrays(scene, dev, refine=levels)
    c = dgs.Camera.from_arrays(cam)
    gpl = np.array([(p << 2) | l for p, l in groups], np.uint16).view(np.int16)
    for tile in ((16, 16), (32, 8)):
        r = dgs.Renderer(dev, tile=tile, states_per_group=8)
        r.plan(s, c, basis, 2 * len(ctx))
        r.bin(s, c, basis)
        delta = r.utility(s, c, _dev(ctx), _dev(cg), _dev(gpl), basis, _dev(ref), BG).cpu().numpy()
        assert r.utility_check() > 0
        mg = ctx.copy()
        for j in range(len(ctx)):
            p, l = groups[cg[j]]
            mg[j, p] = l + 1
        both = r.render(s, c, _dev(np.concatenate([ctx, mg])), basis, BG)
        d = dgs.distortion(both, _dev(ref)).double().cpu().numpy()
        full = d[: len(ctx)] - d[len(ctx):]
        assert np.abs(delta - full).max() <= 1e-6, (tile, np.abs(delta - full).max())
        want = np.concatenate([U.deltas(scene, cam, basis, ctx[cg == k], p, l, ref, np.asarray(BG), refine=levels)
                               for k, (p, l) in enumerate(groups)])
        err = np.abs(delta.astype(np.float64) - want)
        assert err.max() <= 1e-5 + 1e-3 * np.abs(want).max(), (tile, err.max(), np.abs(want).max())
        assert np.abs(want).max() > 1e-4
