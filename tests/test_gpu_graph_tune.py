"""HIP-graph capture of the whole path and the autotuner on the GPU."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
BG = (0.25, 0.5, 0.75)


@pytest.fixture(scope="module")
def dev_workload():
    import paper_2606_17212_amd as dgs
    w = synth.make_workload("g4k_128px_16states", background=BG)
    dev = torch.device("cuda:0")
    return (w, dgs.GaussianScene.from_arrays(w.scene, dev), dgs.Camera.from_arrays(w.camera),
            torch.from_numpy(w.codes).to(dev))


def test_graph_replays_equal_eager_every_time(dev_workload):
    import paper_2606_17212_amd as dgs
    w, scene, cam, codes = dev_workload
    r = dgs.Renderer(states_per_group=8)
    eager = r.render(scene, cam, codes, w.basis, BG).clone()
    g = dgs.CapturedRender(r, scene, cam, codes, w.basis, BG)
    other = dgs.Renderer(states_per_group=4)
    for k in range(4):
        out = g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
        # the program's own eager work between replays, on the same and on another renderer
        r.render(scene, cam, codes.flip(0).contiguous(), w.basis, BG)
        other.render(scene, cam, codes[:3].contiguous(), w.basis, BG)
        torch.cuda.synchronize()
    # contents read at replay time: new opacities show up in the next replay
    old = scene.opacity_logit.clone()
    scene.opacity_logit.add_(0.5)
    want = dgs.Renderer(states_per_group=8).render(scene, cam, codes, w.basis, BG)
    out = g.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    scene.opacity_logit.copy_(old)


def test_graph_psnr_replays(dev_workload):
    import paper_2606_17212_amd as dgs
    w, scene, cam, codes = dev_workload
    r = dgs.Renderer(states_per_group=8)
    ref = r.render(scene, cam, torch.ones_like(codes[:1]), w.basis, BG)[0].contiguous()
    eager = r.render_psnr(scene, cam, codes, w.basis, ref, BG).clone()
    g = dgs.CapturedRender(r, scene, cam, codes, w.basis, BG, reference=ref)
    for _ in range(3):
        out = g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
        r.render(scene, cam, codes, w.basis, BG)
        torch.cuda.synchronize()


def test_autotuner_and_memory_probe(dev_workload, tmp_path):
    import paper_2606_17212_amd as dgs
    from paper_2606_17212_amd.autotune import TILES
    w, scene, cam, codes = dev_workload
    at = dgs.Autotuner(str(tmp_path / "tune.json"))
    res = at.tune(scene, cam, codes, w.basis, BG, reps=2)
    assert res.tile in TILES and res.states_per_group in (2, 4, 8, 16, 32) and res.ms > 0
    again = dgs.Autotuner(str(tmp_path / "tune.json")).tune(scene, cam, codes, w.basis, BG)
    assert (again.tile, again.states_per_group, again.persistent) == (res.tile, res.states_per_group, res.persistent)
    r = dgs.Renderer(tile=res.tile, states_per_group=res.states_per_group, persistent=res.persistent)
    r.plan(scene, cam, w.basis, 16)
    per_state = cam.width * cam.height * 12
    budget = r.workspace_bytes(scene, cam, 100, r.capacity) + 100 * per_state + 1000
    b = dgs.Autotuner.max_states(scene, cam, r, upper=4096, budget_bytes=budget)
    assert 95 <= b <= 100
    assert r.workspace_bytes(scene, cam, b, r.capacity) + b * per_state <= budget
