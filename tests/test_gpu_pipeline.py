"""Renders of successive batches overlapped on several streams (StreamPipeline).

Every call is the whole path on a workspace of its own, so its images must
equal a one-stream render of the same codes bit for bit, whatever the depth,
the launch shape or the order in which the calls' kernels interleave; on the
small workload they are also held to the FP64 oracle (within 1e-4 plus its
ambiguity budget), like the one-stream render.
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


def _batches(w, count, states):
    """``count`` different batches of present-and-depth codes (four layers)."""
    P = w.scene.num_packets
    return [synth.make_codes("present_depth", 0.3, 1.0, states, P, 4, index=w.index, stream=20 + k)
            for k in range(count)]


@pytest.mark.parametrize("depth,S,persistent", [(1, 8, False), (2, 8, False), (3, 8, False), (3, 16, True)])
def test_pipeline_equals_one_stream_250k_800px(depth, S, persistent):
    dgs = _dgs()
    dev = torch.device("cuda:0")
    w = synth.make_workload("g250k_800px_64states", background=BG)
    scene, cam = dgs.GaussianScene.from_arrays(w.scene, dev), dgs.Camera.from_arrays(w.camera)
    batches = [torch.from_numpy(c).to(dev) for c in _batches(w, 7, 24)]
    pipe = dgs.StreamPipeline(dev, depth=depth, tile=(16, 16), states_per_group=S, persistent=persistent)
    pipe.plan(scene, cam, w.basis, 24)
    got = [pipe.render(scene, cam, c, w.basis, BG) for c in batches]  # 7 calls: the slots wrap around
    pipe.join()
    pipe.check()
    r = dgs.Renderer(dev, tile=(16, 16), states_per_group=S, persistent=persistent)
    for k, c in enumerate(batches):
        ref = r.render(scene, cam, c, w.basis, BG)
        assert torch.equal(got[k], ref), f"call {k}"
    r.check()


def test_pipeline_reused_outputs_and_caller_stream_order():
    """Caller-owned outputs reused every ``depth`` calls, and codes written on
    the caller's stream just before each call: every call sees its own codes
    and every output holds the last call that used it."""
    dgs = _dgs()
    dev = torch.device("cuda:0")
    w = synth.make_workload("g250k_800px_64states", background=BG, n=60_000)
    scene, cam = dgs.GaussianScene.from_arrays(w.scene, dev), dgs.Camera.from_arrays(w.camera)
    host = _batches(w, 8, 16)
    src = [torch.from_numpy(c).to(dev) for c in host]
    depth = 3
    pipe = dgs.StreamPipeline(dev, depth=depth, tile=(16, 16), states_per_group=8)
    pipe.plan(scene, cam, w.basis, 16)
    outs = [torch.empty((16, cam.height, cam.width, 3), dtype=torch.float32, device=dev) for _ in range(depth)]
    codes = [torch.empty_like(src[0]) for _ in range(len(src))]  # one input buffer per call
    torch.cuda.synchronize()
    for k in range(len(src)):
        codes[k].copy_(src[k])  # on the caller's stream
        pipe.render(scene, cam, codes[k], w.basis, BG, out=outs[k % depth])
    pipe.join()
    pipe.check()
    r = dgs.Renderer(dev, tile=(16, 16), states_per_group=8)
    for k in range(len(src) - depth, len(src)):
        ref = r.render(scene, cam, src[k], w.basis, BG)
        assert torch.equal(outs[k % depth], ref), f"call {k}"


def test_pipeline_small_workload_matches_oracle():
    dgs = _dgs()
    dev = torch.device("cuda:0")
    w = synth.make_workload("g4k_128px_16states", background=BG)
    ref = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background)
    scene, cam = dgs.GaussianScene.from_arrays(w.scene, dev), dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(np.ascontiguousarray(w.codes)).to(dev)
    pipe = dgs.StreamPipeline(dev, depth=2, tile=(16, 16), states_per_group=16)
    got = [pipe.render(scene, cam, codes, w.basis, BG) for _ in range(3)]  # plans on first use
    pipe.join()
    pipe.check()
    for img in got:
        ex = np.abs(img.cpu().numpy().astype(np.float64) - ref["image"]).max(-1) - ref["budget"]
        assert ex.max() <= TOL, f"max excess {ex.max():.3g}"
    assert torch.equal(got[0], got[2]) and torch.equal(got[0], got[1])
