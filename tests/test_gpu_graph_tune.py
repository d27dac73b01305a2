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


def test_training_step_graph_replays_match_eager(dev_workload):
    """Forward + L1 + backward captured in one graph (torch whole-step
    capture through the C ABI): every replay, with eager work of the same
    renderer and synchronisations in between, reproduces the eager
    gradients up to the order of the FP32 atomics."""
    import paper_2606_17212_amd as dgs
    from paper_2606_17212_amd.render import PARAMS
    w, scene, cam, codes = dev_workload
    dev = codes.device
    r = dgs.Renderer(states_per_group=8)
    full = torch.full((1, w.scene.num_packets), 4, dtype=torch.uint8, device=dev)
    target = r.render(scene, cam, full, w.basis, BG)[:1].clone() * 0.9
    params = {k: getattr(scene, k).clone().requires_grad_(True) for k in PARAMS}
    sc = scene.with_params(**params)
    l1 = dgs.L1Loss(dev)

    def it():
        dgs.l1_loss(dgs.render(r, sc, cam, codes, w.basis, BG), target, None, l1).backward()

    it()
    torch.cuda.synchronize()
    ref = {k: p.grad.clone() for k, p in params.items()}
    # the captured step uses its own leaf tensors, never used on the default
    # stream (a leaf whose gradient node was created on another stream and is
    # still alive does not capture cleanly)
    params = {k: getattr(scene, k).clone().requires_grad_(True) for k in PARAMS}
    sc = scene.with_params(**params)
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        for _ in range(2):
            for p in params.values():
                p.grad = None
            it()
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    for p in params.values():
        p.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        it()
    for rep in range(4):
        graph.replay()
        torch.cuda.synchronize()
        for k in PARAMS:
            nb = float(ref[k].norm())
            assert nb > 0 and float((params[k].grad - ref[k]).norm()) <= 1e-5 * nb, (rep, k)
        # eager work on the same renderer (its workspace) between replays
        r.render(scene, cam, codes[:3].contiguous(), w.basis, BG)
        r.check()
    del graph


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
