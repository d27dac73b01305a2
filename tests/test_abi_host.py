"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol ``include/dgs.h`` declares, sizes workspaces, and rejects bad
arguments before touching the device."""

import ctypes
import os
import re
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2606_17212_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libdgs.so not built (run __graft_entry__.build())")
    return _abi, _abi.lib()


def _declared():
    with open(os.path.join(ROOT, "include", "dgs.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(dgs_\w+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported():
    abi, L = _lib()
    decl = _declared()
    assert len(decl) >= 11
    assert sorted(abi.EXPORTS) == decl
    for name in decl:
        assert hasattr(L, name), name
    assert L.dgs_abi_version() == 3
    assert L.dgs_status_string(3) == b"instance capacity exceeded"


def _cam(abi, w=128, h=96):
    c = abi.Camera()
    for k in range(9):
        c.R_cw[k] = 1.0 if k in (0, 4, 8) else 0.0
    c.t_cw[2] = 3.0
    c.fx = c.fy = 100.0
    c.cx, c.cy, c.near_z = w / 2, h / 2, 0.01
    c.width, c.height = w, h
    return c


def test_workspace_bytes_and_sections():
    abi, L = _lib()
    cam = _cam(abi)
    tun = abi.Tuning(16, 16, 16, 0)
    b0 = L.dgs_workspace_bytes(1000, 32, ctypes.byref(cam), ctypes.byref(tun), 16, 0)
    b1 = L.dgs_workspace_bytes(1000, 32, ctypes.byref(cam), ctypes.byref(tun), 16, 100000)
    assert 0 < b0 < b1
    bad = abi.Tuning(8, 8, 16, 0)
    assert L.dgs_workspace_bytes(1000, 32, ctypes.byref(cam), ctypes.byref(bad), 16, 0) == 0
    assert L.dgs_workspace_bytes(-1, 32, ctypes.byref(cam), ctypes.byref(tun), 16, 0) == 0
    for flags, ok in ((abi.TUNE_PERSISTENT, True), (abi.TUNE_GRID, True),
                      (abi.TUNE_PERSISTENT | abi.TUNE_GRID, False), (4, False)):
        t = abi.Tuning(16, 16, 16, flags)
        assert (L.dgs_workspace_bytes(1000, 32, ctypes.byref(cam), ctypes.byref(t), 16, 0) == b0) == ok, flags
    for batch, ok in ((0, True), (128, True), (256, True), (512, True), (64, False), (384, False), (1024, False)):
        t = abi.Tuning(16, 16, 16, 0, batch)
        assert (L.dgs_workspace_bytes(1000, 32, ctypes.byref(cam), ctypes.byref(t), 16, 0) == b0) == ok, batch
    v = abi.WorkspaceView()
    assert L.dgs_workspace_sections(1000, 32, ctypes.byref(cam), ctypes.byref(tun), 16, 100000,
                                    ctypes.byref(v)) == 0
    assert (v.tiles_x, v.tiles_y) == (8, 6)
    offs = [v.rec0, v.rec1, v.rec2, v.rect, v.ranges, v.sorted_ids]
    assert all(o % 256 == 0 and o < b1 for o in offs)
    tun2 = abi.Tuning(32, 8, 16, 0)
    assert L.dgs_workspace_sections(1000, 32, ctypes.byref(cam), ctypes.byref(tun2), 16, 100000,
                                    ctypes.byref(v)) == 0
    assert (v.tiles_x, v.tiles_y) == (4, 12)


def test_invalid_arguments_rejected_before_any_launch():
    abi, L = _lib()
    cam = _cam(abi)
    tun = abi.Tuning(16, 16, 16, 0)
    st = abi.States()
    st.num_states = 1
    st.codes = 4096  # never dereferenced: validation fails first
    sc = abi.Scene(10, 2, 0, 2, 2, *([4096] * 8))
    ws = ctypes.c_void_p(1 << 20)
    # scene NULL
    assert L.dgs_render(None, ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), ws, 1 << 30, 0,
                        ctypes.c_void_p(4096), None, None) == 1
    assert b"scene" in L.dgs_last_error()
    # rank out of range
    bad = abi.Scene(10, 7, 0, 2, 2, *([4096] * 8))
    assert L.dgs_render(ctypes.byref(bad), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), ws,
                        1 << 30, 0, ctypes.c_void_p(4096), None, None) == 1
    # unsupported tile
    t8 = abi.Tuning(8, 8, 16, 0)
    assert L.dgs_render(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(t8), ws,
                        1 << 30, 0, ctypes.c_void_p(4096), None, None) == 5
    # workspace too small
    assert L.dgs_render(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), ws, 16,
                        0, ctypes.c_void_p(4096), None, None) == 2
    # misaligned workspace
    assert L.dgs_render(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun),
                        ctypes.c_void_p((1 << 20) + 4), 1 << 30, 0, ctypes.c_void_p(4096), None, None) == 1
    # capacity beyond 32-bit offsets
    assert L.dgs_render(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), ws,
                        1 << 30, 1 << 33, ctypes.c_void_p(4096), None, None) == 1
    # camera size
    c0 = _cam(abi, 0, 10)
    assert L.dgs_render(ctypes.byref(sc), ctypes.byref(c0), ctypes.byref(st), ctypes.byref(tun), ws,
                        1 << 30, 0, ctypes.c_void_p(4096), None, None) == 1
    # missing image / grads
    assert L.dgs_render(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), ws,
                        1 << 30, 0, None, None, None) == 1
    g = abi.SceneGrad(None, None, None, None, None, None)
    assert L.dgs_backward(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), ws,
                          1 << 30, 0, ctypes.c_void_p(4096), ctypes.c_void_p(4096), ctypes.byref(g),
                          None) == 1


def test_python_binding_validates_tensors():
    import torch

    import paper_2606_17212_amd as dgs
    from paper_2606_17212_amd.render import _c_scene
    sc = dgs.GaussianScene(torch.zeros(3, 5), torch.zeros(3, 5), torch.zeros(4, 5), torch.zeros(5),
                           torch.zeros(3, 5), torch.zeros(6, 5), torch.zeros(5, dtype=torch.int16),
                           2, 2, 2, 0)
    _c_scene(sc)  # shapes and dtypes fine (host tensors: pointers are only marshalled)
    with pytest.raises(ValueError):
        _c_scene(sc.with_params(color=torch.zeros(12, 5)))
    with pytest.raises(TypeError):
        _c_scene(sc.with_params(mean=torch.zeros(3, 5, dtype=torch.float64)))


def test_loss_entry_points_validate_before_any_launch():
    """L1 loss and Eq. (2) objective: sizes and pointers are checked on the
    host (no device pointer is touched when a check fails)."""
    abi, L = _lib()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced
    assert L.dgs_l1_scratch_bytes(8, 1280, 720) > 0
    assert L.dgs_l1_scratch_bytes(-1, 16, 16) == 0 and L.dgs_l1_scratch_bytes(1, 0, 16) == 0
    assert L.dgs_l1_scratch_bytes(65536, 16, 16) == 0
    need = L.dgs_l1_scratch_bytes(2, 16, 16)
    loss = ctypes.c_void_p(1 << 21)
    # bad sizes, missing targets, missing loss / scratch, misaligned or short scratch
    assert L.dgs_l1_loss(fake, -1, 16, 16, fake, 1, None, loss, fake, need, None) == 1
    assert L.dgs_l1_loss(fake, 2, 0, 16, fake, 1, None, loss, fake, need, None) == 1
    assert L.dgs_l1_loss(fake, 2, 16, 16, None, 1, None, loss, fake, need, None) == 1
    assert L.dgs_l1_loss(fake, 2, 16, 16, fake, 0, None, loss, fake, need, None) == 1
    assert L.dgs_l1_loss(fake, 2, 16, 16, fake, 1, None, None, fake, need, None) == 1
    assert L.dgs_l1_loss(fake, 2, 16, 16, fake, 1, None, loss, None, need, None) == 1
    assert L.dgs_l1_loss(fake, 2, 16, 16, fake, 1, None, loss, ctypes.c_void_p((1 << 20) + 4), need, None) == 1
    assert b"aligned" in L.dgs_last_error()
    assert L.dgs_l1_loss(fake, 2, 16, 16, fake, 1, None, loss, fake, need - 1, None) == 2
    assert L.dgs_l1_loss_grad(fake, 2, 16, 16, fake, 1, None, None, None, None) == 1
    assert b"grad" in L.dgs_last_error()
    # objective: alpha outside (0, 1] and negative weights are refused
    w = abi.ObjectiveWeights(0.2, 0.3, 0.0, 0.1, 2.0, 0.5)
    ob = L.dgs_objective_scratch_bytes(2, 16, 16, 0)
    assert ob > 0
    assert L.dgs_objective(fake, 2, 16, 16, fake, 1, fake, fake, 1, None, 0, None, 0, None, 0, ctypes.byref(w),
                           loss, None, None, fake, ob, None) == 1
    w = abi.ObjectiveWeights(0.2, -0.3, 0.05, 0.1, 2.0, 0.5)
    assert L.dgs_objective(fake, 2, 16, 16, fake, 1, fake, fake, 1, None, 0, None, 0, None, 0, ctypes.byref(w),
                           loss, None, None, fake, ob, None) == 1


def test_count_instances_null_states_and_near_plane_rejected():
    abi, L = _lib()
    cam = _cam(abi)
    tun = abi.Tuning(16, 16, 16, 0)
    st = abi.States()
    sc = abi.Scene(10, 2, 0, 2, 2, *([4096] * 8))
    ws = ctypes.c_void_p(1 << 20)
    m = ctypes.c_int64(0)
    assert L.dgs_count_instances(ctypes.byref(sc), ctypes.byref(cam), None, ctypes.byref(tun), ws, 1 << 30,
                                 ctypes.byref(m), None) == 1
    assert b"states" in L.dgs_last_error()
    for near in (0.0, -0.5):
        c = _cam(abi)
        c.near_z = near
        assert L.dgs_count_instances(ctypes.byref(sc), ctypes.byref(c), ctypes.byref(st), ctypes.byref(tun), ws,
                                     1 << 30, ctypes.byref(m), None) == 1
        assert b"near_z" in L.dgs_last_error()
        assert L.dgs_workspace_bytes(1000, 4, ctypes.byref(c), ctypes.byref(tun), 16, 0) == 0


def _capturing(monkeypatch):
    import torch
    monkeypatch.setattr(torch.cuda, "is_available", lambda: True)
    monkeypatch.setattr(torch.cuda, "is_current_stream_capturing", lambda: True)


def test_python_synchronising_calls_refuse_graph_capture(monkeypatch):
    """Every binding call that waits for the device raises, before any
    device work, while the current stream is being captured."""
    import torch

    import paper_2606_17212_amd as dgs
    from paper_2606_17212_amd.render import PARAMS, RenderFunction
    _capturing(monkeypatch)
    r = dgs.Renderer(torch.device("cuda", 0))
    sc = dgs.GaussianScene(torch.zeros(3, 5), torch.zeros(3, 5), torch.zeros(4, 5), torch.zeros(5),
                           torch.zeros(3, 5), torch.zeros(6, 5), torch.zeros(5, dtype=torch.int16), 2, 2, 2, 0)
    cam = dgs.Camera([1, 0, 0, 0, 1, 0, 0, 0, 1], [0, 0, 3], 100.0, 100.0, 32.0, 32.0, 64, 64)
    codes = torch.zeros(2, 4, dtype=torch.uint8)
    calls = [lambda: r.plan(sc, cam, [0.5, 0.25], 2), lambda: r.count_instances(sc, cam, [0.5, 0.25]),
             lambda: r.check(), lambda: r.sections(sc, cam, 2), lambda: r.composite_stats(sc, cam, codes, [0, 0]),
             lambda: r.utility_items(sc, cam, codes, None, None, [0, 0]), lambda: r.utility_check(),
             lambda: dgs.Objective(torch.device("cuda", 0)).check(),
             lambda: dgs.L1Loss(torch.device("cuda", 0)).check()]
    for f in calls:
        with pytest.raises(RuntimeError, match="captured"):
            f()

    # a backward whose forward's lists were overwritten by another render
    ctx = SimpleNamespace(renderer=r, scene=sc, camera=cam, codes=codes, basis=(0.5, 0.25), background=(0, 0, 0),
                          generation=r.generation - 1,
                          saved_tensors=(torch.zeros(2, 64, 64, 3),) + tuple(getattr(sc, k) for k in PARAMS))
    with pytest.raises(RuntimeError, match="re-render"):
        RenderFunction.backward(ctx, torch.zeros(2, 64, 64, 3))


def test_live_capture_blocks_replanning(monkeypatch):
    """While a captured graph holds pointers into a renderer's workspace,
    planning again or growing the workspace raises."""
    import torch

    import paper_2606_17212_amd as dgs
    r = dgs.Renderer(torch.device("cuda", 0))
    r.ws = torch.zeros(1024, dtype=torch.uint8)
    r.ws_bytes = 1024
    r.live_captures = 1
    sc = dgs.GaussianScene(torch.zeros(3, 5), torch.zeros(3, 5), torch.zeros(4, 5), torch.zeros(5),
                           torch.zeros(3, 5), torch.zeros(6, 5), torch.zeros(5, dtype=torch.int16), 2, 2, 2, 0)
    cam = dgs.Camera([1, 0, 0, 0, 1, 0, 0, 0, 1], [0, 0, 3], 100.0, 100.0, 32.0, 32.0, 64, 64)
    with pytest.raises(RuntimeError, match="close"):
        r.plan(sc, cam, [0.5, 0.25], 4)
    with pytest.raises(RuntimeError, match="close"):
        r._ensure_ws(4096)
    r._ensure_ws(512)  # fits: the buffer is kept
    assert r.ws_bytes == 1024


def test_noalloc_render_refuses_oversize_and_bad_arguments_before_any_hip_call():
    """dgs_render_noalloc: a call whose workspace would not fit the static
    array, and malformed arguments, are refused on the host."""
    abi, L = _lib()
    cam = _cam(abi)
    tun = abi.Tuning(16, 16, 16, 0)
    st = abi.States()
    st.num_states = 16
    st.codes = 4096  # never dereferenced
    img = ctypes.c_void_p(4096)
    sc = abi.Scene(4096, 2, 0, 8, 4, *([4096] * 8))
    need = L.dgs_workspace_bytes(4096, 32, ctypes.byref(cam), ctypes.byref(tun), 16, 200_000)
    assert 0 < need <= abi.NOALLOC_SCRATCH_BYTES
    # the instance capacity alone pushes the workspace past the array
    big = 0xFFFFFFFF
    assert L.dgs_workspace_bytes(4096, 32, ctypes.byref(cam), ctypes.byref(tun), 16, big) > \
        abi.NOALLOC_SCRATCH_BYTES
    assert L.dgs_render_noalloc(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), big,
                                img, None, None, None) == 2
    assert b"static scratch" in L.dgs_last_error()
    # so does a large scene
    sc_big = abi.Scene(4_000_000, 2, 0, 8, 4, *([4096] * 8))
    assert L.dgs_render_noalloc(ctypes.byref(sc_big), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun),
                                1000, img, None, None, None) == 2
    # missing image, NULL scene, bad capacity, unsupported tile
    assert L.dgs_render_noalloc(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), 1000,
                                None, None, None, None) == 1
    assert L.dgs_render_noalloc(None, ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), 1000, img, None,
                                None, None) == 1
    assert L.dgs_render_noalloc(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(tun), -1, img,
                                None, None, None) == 1
    t8 = abi.Tuning(8, 8, 16, 0)
    assert L.dgs_render_noalloc(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(st), ctypes.byref(t8), 1000,
                                img, None, None, None) == 5


def test_stream_pipeline_rejects_a_depth_below_one_before_touching_the_device():
    import paper_2606_17212_amd as dgs
    for depth in (0, -2):
        with pytest.raises(ValueError, match="depth"):
            dgs.StreamPipeline("cuda", depth=depth)
