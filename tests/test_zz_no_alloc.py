"""dgs_render_noalloc (the render whose workspace is the library's static
device array) against dgs_render with a caller-owned workspace, through the
C ABI: two calls in a row, the second with a smaller input (fewer Gaussians,
fewer states, a smaller camera), each bit-identical to dgs_render in images,
T_final and the instance count."""

import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
BG = (0.25, 0.5, 0.75)


def _bind():
    import importlib
    from paper_2606_17212_amd import _abi
    return _abi, importlib.import_module("paper_2606_17212_amd.render")


def _subset(scene, n):
    keys = ("mean", "log_scale", "quat", "color", "temporal")
    p = {k: getattr(scene, k)[:, :n].contiguous() for k in keys}
    p["opacity_logit"] = scene.opacity_logit[:n].contiguous()
    p["packet_layer"] = scene.packet_layer[:n].contiguous()
    return scene.with_params(**p)


def _args(render, scene, cam, codes, basis, tun):
    return (render._c_scene(scene), render._c_camera(cam), render._c_states(codes, basis, BG), tun)


def _with_workspace(abi, render, scene, cam, codes, basis, tun, cap, dev):
    L = abi.lib()
    sc, cc, st, tu = _args(render, scene, cam, codes, basis, tun)
    W = int(codes.shape[0])
    nbytes = L.dgs_workspace_bytes(scene.records, scene.num_packets, ctypes.byref(cc), ctypes.byref(tu), W, cap)
    assert nbytes > 0
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
    img = torch.empty((W, cam.height, cam.width, 3), dtype=torch.float32, device=dev)
    tf = torch.empty((W, cam.height, cam.width), dtype=torch.float32, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    abi.check(L.dgs_render(ctypes.byref(sc), ctypes.byref(cc), ctypes.byref(st), ctypes.byref(tu),
                           ctypes.c_void_p(ws.data_ptr()), int(nbytes), cap, ctypes.c_void_p(img.data_ptr()),
                           ctypes.c_void_p(tf.data_ptr()), stream))
    m = ctypes.c_int64(0)
    abi.check(L.dgs_check(ctypes.c_void_p(ws.data_ptr()), int(nbytes), ctypes.byref(m), stream))
    return img, tf, int(m.value), int(nbytes)


def _noalloc(abi, render, scene, cam, codes, basis, tun, cap, dev):
    L = abi.lib()
    sc, cc, st, tu = _args(render, scene, cam, codes, basis, tun)
    W = int(codes.shape[0])
    # outputs start as NaN / -1 so that anything the call leaves unwritten shows
    img = torch.full((W, cam.height, cam.width, 3), float("nan"), dtype=torch.float32, device=dev)
    tf = torch.full((W, cam.height, cam.width), float("nan"), dtype=torch.float32, device=dev)
    inst = torch.full((1,), -1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize(dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    abi.check(L.dgs_render_noalloc(ctypes.byref(sc), ctypes.byref(cc), ctypes.byref(st), ctypes.byref(tu), cap,
                                   ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(tf.data_ptr()),
                                   ctypes.c_void_p(inst.data_ptr()), stream))
    torch.cuda.synchronize(dev)
    return img, tf, int(inst.item())


def _smaller_camera(cam, width, height):
    from dataclasses import replace
    return replace(cam, width=width, height=height, cx=cam.cx * width / cam.width, cy=cam.cy * height / cam.height)


def test_noalloc_equals_render_two_calls_second_smaller():
    import paper_2606_17212_amd as dgs
    abi, render = _bind()
    dev = torch.device("cuda:0")
    w = synth.make_workload("g4k_128px_16states", background=BG)
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(np.ascontiguousarray(w.codes)).to(dev)
    tun = abi.Tuning(16, 16, 8, 0, 256)
    cap = 200_000
    # 1: the 4,096-Gaussian 128x128 workload, 16 states
    print(f"[noalloc] call 1: n={scene.n} {cam.width}x{cam.height} W={codes.shape[0]}", flush=True)
    ref_img, ref_tf, ref_m, nbytes = _with_workspace(abi, render, scene, cam, codes, w.basis, tun, cap, dev)
    assert 0 < ref_m <= cap and nbytes <= abi.NOALLOC_SCRATCH_BYTES
    img, tf, m = _noalloc(abi, render, scene, cam, codes, w.basis, tun, cap, dev)
    assert m == ref_m
    assert torch.equal(img, ref_img) and torch.equal(tf, ref_tf)
    # 2: a smaller input right after: 1,500 Gaussians, 5 states, a 96x80 camera, 32x8 tiles
    small = _subset(scene, 1500)
    scam = _smaller_camera(cam, 96, 80)
    scodes = codes[3:8].contiguous()
    stun = abi.Tuning(32, 8, 4, 0, 256)
    print(f"[noalloc] call 2: n={small.n} {scam.width}x{scam.height} W={scodes.shape[0]}", flush=True)
    ref_img2, ref_tf2, ref_m2, _ = _with_workspace(abi, render, small, scam, scodes, w.basis, stun, cap, dev)
    img2, tf2, m2 = _noalloc(abi, render, small, scam, scodes, w.basis, stun, cap, dev)
    assert 0 < ref_m2 < ref_m and m2 == ref_m2
    assert torch.equal(img2, ref_img2) and torch.equal(tf2, ref_tf2)
    assert torch.isfinite(img2).all()


def test_noalloc_python_binding_and_limits():
    import paper_2606_17212_amd as dgs
    abi, render = _bind()
    dev = torch.device("cuda:0")
    w = synth.make_workload("g4k_128px_16states", background=BG)
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(np.ascontiguousarray(w.codes)).to(dev)
    r = dgs.Renderer(dev, tile=(16, 16), states_per_group=16)
    ref = r.render(scene, cam, codes, w.basis, BG)
    m = r.check()
    out = torch.empty_like(ref)
    inst = torch.zeros(1, dtype=torch.int64, device=dev)
    print("[noalloc] python binding, 16 states", flush=True)
    dgs.render_noalloc(scene, cam, codes, w.basis, BG, r.capacity, out, instances=inst, states_per_group=16)
    torch.cuda.synchronize(dev)
    assert torch.equal(out, ref) and int(inst.item()) == m
    # a capacity too small for the scene: the count says so (the images are undefined then)
    print("[noalloc] capacity below the instance count", flush=True)
    dgs.render_noalloc(scene, cam, codes, w.basis, BG, m // 2, out, instances=inst, states_per_group=16)
    torch.cuda.synchronize(dev)
    assert int(inst.item()) == m
    # a call whose workspace exceeds the static array is refused before any launch
    huge = 0xFFFFFFFF
    with pytest.raises(abi.DgsError) as e:
        dgs.render_noalloc(scene, cam, codes, w.basis, BG, huge, out)
    assert e.value.status == 2 and "static scratch" in str(e.value)
    # and a normal call afterwards is still exact
    dgs.render_noalloc(scene, cam, codes, w.basis, BG, r.capacity, out, states_per_group=16)
    torch.cuda.synchronize(dev)
    assert torch.equal(out, ref)
