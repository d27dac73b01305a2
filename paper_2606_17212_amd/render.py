"""Python binding of the renderer: device tensors in, device tensors out.

PyTorch provides device memory and the stream; every step of the render runs
in the HIP kernels of ``libdgs.so`` through the C ABI (``_abi``).  The
binding marshals arguments and sizes the caller-owned workspace.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi

PARAMS = ("mean", "log_scale", "quat", "opacity_logit", "color", "temporal")


@dataclass
class GaussianScene:
    """Scene on the device (FP32 component-major arrays, see include/dgs.h)."""
    mean: torch.Tensor
    log_scale: torch.Tensor
    quat: torch.Tensor
    opacity_logit: torch.Tensor
    color: torch.Tensor
    temporal: torch.Tensor
    packet_layer: torch.Tensor  # int16 storage of the uint16 (packet << 2) | layer
    num_clusters: int
    num_contexts: int
    rank: int
    sh_degree: int
    cluster_affine: Optional[torch.Tensor] = None
    # [3][rows][n] refinement levels (position residual 3, log-scale 3,
    # quaternion 4, opacity logit 1, colour 3 or 12), or None
    refine: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @property
    def records(self) -> int:
        """Projected records: one per Gaussian, or one per (Gaussian,
        delivered depth) with refinement levels."""
        return self.n * (4 if self.refine is not None else 1)

    @property
    def num_packets(self) -> int:
        return self.num_clusters * self.num_contexts

    @staticmethod
    def from_arrays(a, device="cuda", refine=None) -> "GaussianScene":
        """From a host container with numpy fields of the same names;
        ``refine``: optional host array of refinement levels [3][rows][n]."""
        import numpy as np

        t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device)  # noqa: E731
        pl = torch.from_numpy(np.ascontiguousarray(a.packet_layer, dtype=np.uint16).view(np.int16)).to(device)
        aff = None if a.cluster_affine is None else t(a.cluster_affine)
        return GaussianScene(t(a.mean), t(a.log_scale), t(a.quat), t(a.opacity_logit), t(a.color),
                             t(a.temporal), pl, a.num_clusters, a.num_contexts, a.rank, a.sh_degree, aff,
                             None if refine is None else t(refine))

    def with_params(self, **p) -> "GaussianScene":
        d = dict(self.__dict__)
        d.update(p)
        return GaussianScene(**d)


@dataclass
class Camera:
    R_cw: Sequence[float]  # 9 floats, row-major
    t_cw: Sequence[float]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.01

    @staticmethod
    def from_arrays(c) -> "Camera":
        import numpy as np
        return Camera([float(x) for x in np.asarray(c.R_cw, np.float32).reshape(9)],
                      [float(x) for x in np.asarray(c.t_cw, np.float32).reshape(3)],
                      c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.near)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_tensor(t, name, dtype, device):
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")


def _refuse_capture(what: str, device=None):
    """Calls that wait for the device (a header copied to the host, a
    synchronisation, an allocation-sized plan) cannot be recorded in a HIP
    graph; refuse them with a clear error while the current stream captures."""
    if torch.cuda.is_available() and torch.cuda.is_current_stream_capturing():
        raise RuntimeError(f"{what} synchronises with the host and cannot run while the current stream is "
                           "being captured into a graph; call it before the capture")


def _c_scene(s: GaussianScene, params=None) -> _abi.Scene:
    p = params or {k: getattr(s, k) for k in PARAMS}
    dev = p["mean"].device
    for k in PARAMS:
        _check_tensor(p[k], k, torch.float32, dev)
    _check_tensor(s.packet_layer, "packet_layer", torch.int16, dev)
    n = s.n
    shapes = dict(mean=(3, n), log_scale=(3, n), quat=(4, n), opacity_logit=(n,),
                  color=((3 if s.sh_degree == 0 else 12), n), temporal=(3 * s.rank, n))
    for k, shp in shapes.items():
        if tuple(p[k].shape) != shp:
            raise ValueError(f"{k} has shape {tuple(p[k].shape)}, expected {shp}")
    if s.cluster_affine is not None:
        _check_tensor(s.cluster_affine, "cluster_affine", torch.float32, dev)
        if s.cluster_affine.numel() != 12 * s.num_clusters or s.cluster_affine.shape[0] != s.num_clusters:
            raise ValueError(f"cluster_affine has shape {tuple(s.cluster_affine.shape)}, "
                             f"expected ({s.num_clusters}, 12) or ({s.num_clusters}, 3, 4)")
    if s.refine is not None:
        _check_tensor(s.refine, "refine", torch.float32, dev)
        shp = (3, 11 + (3 if s.sh_degree == 0 else 12), n)
        if tuple(s.refine.shape) != shp:
            raise ValueError(f"refine has shape {tuple(s.refine.shape)}, expected {shp}")
    return _abi.Scene(n, s.rank, s.sh_degree, s.num_clusters, s.num_contexts, _ptr(p["mean"]),
                      _ptr(p["log_scale"]), _ptr(p["quat"]), _ptr(p["opacity_logit"]), _ptr(p["color"]),
                      _ptr(p["temporal"]), _ptr(s.packet_layer), _ptr(s.cluster_affine), _ptr(s.refine))


def _c_camera(c: Camera) -> _abi.Camera:
    cc = _abi.Camera()
    for k in range(9):
        cc.R_cw[k] = float(c.R_cw[k])
    for k in range(3):
        cc.t_cw[k] = float(c.t_cw[k])
    cc.fx, cc.fy, cc.cx, cc.cy, cc.near_z = c.fx, c.fy, c.cx, c.cy, c.near
    cc.width, cc.height = int(c.width), int(c.height)
    return cc


def _c_states(codes: Optional[torch.Tensor], basis, background, num_states=None) -> _abi.States:
    st = _abi.States()
    st.num_states = int(codes.shape[0]) if codes is not None else int(num_states or 0)
    st.codes = _ptr(codes)
    b = list(basis) + [0.0] * (4 - len(basis))
    for k in range(4):
        st.basis[k] = float(b[k])
    for k in range(3):
        st.background[k] = float(background[k])
    return st


def render_noalloc(scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis, background,
                   instance_capacity: int, out: torch.Tensor, tfinal: Optional[torch.Tensor] = None,
                   instances: Optional[torch.Tensor] = None, tile=(16, 16), states_per_group=16,
                   persistent=None, lds_batch=256) -> torch.Tensor:
    """``dgs_render_noalloc``: a batched render whose workspace is the
    library's static device array, for callers that cannot allocate (graph
    capture, serving loops).  Every output is caller-provided: ``out`` [W, H,
    Wd, 3] FP32, optional ``tfinal`` [W, H, Wd] FP32 and ``instances`` int64
    [1] (the tile instances the scene needs; above ``instance_capacity`` the
    images are undefined).  Raises DgsError (DGS_ERR_WORKSPACE) when the call
    does not fit the array (``DGS_NOALLOC_SCRATCH_BYTES``).  Calls on one GPU
    share the array and must not overlap."""
    dev = out.device
    _check_tensor(codes, "codes", torch.uint8, dev)
    if codes.dim() != 2 or codes.shape[1] != scene.num_packets:
        raise ValueError(f"codes must be [W, {scene.num_packets}]")
    W = int(codes.shape[0])
    _check_tensor(out, "out", torch.float32, dev)
    if tuple(out.shape) != (W, camera.height, camera.width, 3):
        raise ValueError(f"out has shape {tuple(out.shape)}, expected {(W, camera.height, camera.width, 3)}")
    if tfinal is not None:
        _check_tensor(tfinal, "tfinal", torch.float32, dev)
        if tuple(tfinal.shape) != (W, camera.height, camera.width):
            raise ValueError(f"tfinal has shape {tuple(tfinal.shape)}, expected {(W, camera.height, camera.width)}")
    if instances is not None:
        _check_tensor(instances, "instances", torch.int64, dev)
        if instances.numel() < 1:
            raise ValueError("instances needs one element")
    flags = 0 if persistent is None else (_abi.TUNE_PERSISTENT if persistent else _abi.TUNE_GRID)
    tun = _abi.Tuning(int(tile[0]), int(tile[1]), int(states_per_group), flags, int(lds_batch))
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _abi.check(_abi.lib().dgs_render_noalloc(
        ctypes.byref(_c_scene(scene)), ctypes.byref(_c_camera(camera)),
        ctypes.byref(_c_states(codes, basis, background)), ctypes.byref(tun), int(instance_capacity),
        _ptr(out), _ptr(tfinal), _ptr(instances), st))
    return out


class Renderer:
    """Owns the device workspace and the launch shape.

    ``plan`` counts the scene's tile instances (one synchronisation) and sizes
    the workspace; ``render`` and friends are then asynchronous on the
    current stream.  ``slack`` over-provisions the instance capacity so a
    scene whose parameters change (training) rarely needs a new plan;
    ``check()`` reports an overflow.
    """

    def __init__(self, device="cuda", tile=(16, 16), states_per_group=16, slack=1.25, persistent=None,
                 lds_batch=256):
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        # compositing launch: True persistent, False grid, None chosen by the library
        flags = 0 if persistent is None else (_abi.TUNE_PERSISTENT if persistent else _abi.TUNE_GRID)
        # list entries staged in LDS per batch (128, 256 or 512; images do not depend on it)
        self.tuning = _abi.Tuning(int(tile[0]), int(tile[1]), int(states_per_group), flags, int(lds_batch))
        self.slack = float(slack)
        self.ws = None
        self.ws_bytes = 0
        self.capacity = 0
        self.max_states = 0
        self.generation = 0  # bumps whenever the workspace's sorted lists change
        self.uws = None       # utility workspace
        self.utility_capacity = 0
        self._key = None
        self.live_captures = 0  # CapturedRender graphs holding pointers into the workspace

    # ---------------------------------------------------------------- planning
    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _ensure_ws(self, nbytes):
        if self.ws is None or self.ws_bytes < nbytes:
            if self.live_captures:
                raise RuntimeError(f"the workspace must grow to {int(nbytes)} bytes, but {self.live_captures} "
                                   "captured graph(s) hold pointers into it; close() them first")
            # 256-byte aligned device buffer (torch's caching allocator aligns to 512)
            self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            self.ws_bytes = int(nbytes)

    def workspace_bytes(self, scene: GaussianScene, camera: Camera, max_states: int, capacity: int) -> int:
        b = _abi.lib().dgs_workspace_bytes(scene.records, scene.num_packets, ctypes.byref(_c_camera(camera)),
                                           ctypes.byref(self.tuning), int(max_states), int(capacity))
        if b == 0:
            raise ValueError("invalid arguments for dgs_workspace_bytes: "
                             + _abi.lib().dgs_last_error().decode())
        return int(b)

    def count_instances(self, scene: GaussianScene, camera: Camera, basis, params=None) -> int:
        _refuse_capture("Renderer.count_instances")
        L = _abi.lib()
        cam = _c_camera(camera)
        self._ensure_ws(self.workspace_bytes(scene, camera, 0, 0))
        m = ctypes.c_int64(0)
        st = _c_states(None, basis, (0, 0, 0))
        _abi.check(L.dgs_count_instances(ctypes.byref(_c_scene(scene, params)), ctypes.byref(cam),
                                         ctypes.byref(st), ctypes.byref(self.tuning), _ptr(self.ws),
                                         self.ws_bytes, ctypes.byref(m), self._stream()))
        self.generation += 1
        return int(m.value)

    def plan(self, scene: GaussianScene, camera: Camera, basis, max_states: int, params=None) -> int:
        _refuse_capture("Renderer.plan")
        if self.live_captures:
            raise RuntimeError(f"{self.live_captures} captured graph(s) hold pointers into this renderer's "
                               "workspace and capacity; close() them before planning again")
        m = self.count_instances(scene, camera, basis, params)
        cap = max(int(m * self.slack) + 1024, 1024)
        cap = min(cap, 0xFFFFFFFF)
        self.capacity = cap
        self.max_states = int(max_states)
        self._ensure_ws(self.workspace_bytes(scene, camera, max_states, cap))
        self._key = (scene.records, camera.width, camera.height)
        return m

    def _need_plan(self, scene, camera, basis, W, params=None):
        if self._key != (scene.records, camera.width, camera.height) or W > self.max_states or self.capacity == 0:
            self.plan(scene, camera, basis, max(W, self.max_states), params)

    def sections(self, scene: GaussianScene, camera: Camera, num_states: int) -> dict:
        """Intermediate results of the last render (synchronises): per-record
        data and rectangles, per-tile ranges and the sorted ids."""
        _refuse_capture("Renderer.sections")
        v = _abi.WorkspaceView()
        _abi.check(_abi.lib().dgs_workspace_sections(
            scene.records, scene.num_packets, ctypes.byref(_c_camera(camera)), ctypes.byref(self.tuning),
            int(num_states), self.capacity, ctypes.byref(v)))
        torch.cuda.synchronize(self.device)
        n, tiles = scene.records, v.tiles_x * v.tiles_y

        def sl(off, count, dtype, width):
            nbytes = count * width * torch.tensor([], dtype=dtype).element_size()
            return self.ws[off:off + nbytes].view(dtype).reshape(count, width).cpu()

        return dict(rec0=sl(v.rec0, n, torch.float32, 4), rec1=sl(v.rec1, n, torch.float32, 4),
                    rec2=sl(v.rec2, n, torch.float32, 4), rect=sl(v.rect, n, torch.int32, 2),
                    ranges=sl(v.ranges, tiles, torch.int32, 2),
                    # sorted values: Gaussian id in bits 0..27, wave-block reach mask in bits 28..31
                    sorted_ids=sl(v.sorted_ids, self.capacity, torch.int32, 1).reshape(-1) & 0x0FFFFFFF,
                    wave_masks=(sl(v.sorted_ids, self.capacity, torch.int32, 1).reshape(-1) >> 28) & 0xF,
                    tiles_x=v.tiles_x, tiles_y=v.tiles_y)

    def check(self) -> int:
        """Synchronise and return the last binning's instance count; raises
        DgsError on overflow."""
        _refuse_capture("Renderer.check")
        m = ctypes.c_int64(0)
        _abi.check(_abi.lib().dgs_check(_ptr(self.ws), self.ws_bytes, ctypes.byref(m), self._stream()))
        return int(m.value)

    # ------------------------------------------------------------------ calls
    def _codes(self, codes, scene):
        _check_tensor(codes, "codes", torch.uint8, self.device)
        if codes.dim() != 2 or codes.shape[1] != scene.num_packets:
            raise ValueError(f"codes must be [W, {scene.num_packets}]")

    def render(self, scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis, background=(0, 0, 0),
               tfinal: bool = False, params=None, per_state: bool = False, out=None):
        """Images [W, H, Wd, 3] (and T_final [W, H, Wd] when ``tfinal``)."""
        self._codes(codes, scene)
        W = int(codes.shape[0])
        self._need_plan(scene, camera, basis, W, params)
        img = out if out is not None else torch.empty((W, camera.height, camera.width, 3),
                                                      dtype=torch.float32, device=self.device)
        tf = torch.empty((W, camera.height, camera.width), dtype=torch.float32,
                         device=self.device) if tfinal else None
        fn = _abi.lib().dgs_render_per_state if per_state else _abi.lib().dgs_render
        _abi.check(fn(ctypes.byref(_c_scene(scene, params)), ctypes.byref(_c_camera(camera)),
                      ctypes.byref(_c_states(codes, basis, background)), ctypes.byref(self.tuning),
                      _ptr(self.ws), self.ws_bytes, self.capacity, _ptr(img), _ptr(tf), self._stream()))
        self.generation += 1
        return (img, tf) if tfinal else img

    def bin(self, scene: GaussianScene, camera: Camera, basis, params=None):
        """Shared half of a render: projection, depth sort, tile lists."""
        self._need_plan(scene, camera, basis, self.max_states, params)
        _abi.check(_abi.lib().dgs_bin(
            ctypes.byref(_c_scene(scene, params)), ctypes.byref(_c_camera(camera)),
            ctypes.byref(_c_states(None, basis, (0, 0, 0))), ctypes.byref(self.tuning), _ptr(self.ws),
            self.ws_bytes, self.capacity, self._stream()))
        self.generation += 1

    def composite(self, scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis, background=(0, 0, 0),
                  tfinal: bool = False, out=None):
        """Masked compositing of every state in ``codes`` from the last ``bin``."""
        self._codes(codes, scene)
        W = int(codes.shape[0])
        if W > self.max_states:
            raise ValueError(f"{W} states > planned {self.max_states}; plan again")
        img = out if out is not None else torch.empty((W, camera.height, camera.width, 3),
                                                      dtype=torch.float32, device=self.device)
        tf = torch.empty((W, camera.height, camera.width), dtype=torch.float32,
                         device=self.device) if tfinal else None
        _abi.check(_abi.lib().dgs_composite(
            ctypes.byref(_c_scene(scene)), ctypes.byref(_c_camera(camera)),
            ctypes.byref(_c_states(codes, basis, background)), ctypes.byref(self.tuning), _ptr(self.ws),
            self.ws_bytes, self.capacity, _ptr(img), _ptr(tf), self._stream()))
        return (img, tf) if tfinal else img

    def composite_psnr(self, scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis,
                       reference: torch.Tensor, background=(0, 0, 0), out=None):
        """PSNR [W] from the last ``bin`` (no image written)."""
        self._codes(codes, scene)
        _check_tensor(reference, "reference", torch.float32, self.device)
        W = int(codes.shape[0])
        if W > self.max_states:
            raise ValueError(f"{W} states > planned {self.max_states}; plan again")
        ps = out if out is not None else torch.empty((W,), dtype=torch.float32, device=self.device)
        _abi.check(_abi.lib().dgs_composite_psnr(
            ctypes.byref(_c_scene(scene)), ctypes.byref(_c_camera(camera)),
            ctypes.byref(_c_states(codes, basis, background)), ctypes.byref(self.tuning), _ptr(self.ws),
            self.ws_bytes, self.capacity, _ptr(reference), _ptr(ps), self._stream()))
        return ps

    def composite_stats(self, scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis):
        """(alpha evaluations, blends, wave evaluations, wave misses) one
        ``composite`` of ``codes`` performs after the last ``bin`` (synchronises)."""
        _refuse_capture("Renderer.composite_stats")
        self._codes(codes, scene)
        cnt = torch.zeros(4, dtype=torch.int64, device=self.device)
        _abi.check(_abi.lib().dgs_composite_stats(
            ctypes.byref(_c_scene(scene)), ctypes.byref(_c_camera(camera)),
            ctypes.byref(_c_states(codes, basis, (0, 0, 0))), ctypes.byref(self.tuning), _ptr(self.ws),
            self.ws_bytes, self.capacity, _ptr(cnt), self._stream()))
        return tuple(int(x) for x in cnt.cpu().tolist())

    def launch_plan(self, camera: Camera, num_states: int):
        """How ``composite`` launches for ``num_states`` states: dict with
        ``states_per_group``, ``persistent``, ``workgroups``, ``work_items``,
        ``lds_batch``."""
        with torch.cuda.device(self.device):
            S, pers = ctypes.c_int32(), ctypes.c_int32()
            wg, items, lb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
            _abi.check(_abi.lib().dgs_composite_launch(ctypes.byref(_c_camera(camera)), ctypes.byref(self.tuning),
                                                       int(num_states), ctypes.byref(S), ctypes.byref(pers),
                                                       ctypes.byref(wg), ctypes.byref(items), ctypes.byref(lb)))
        return {"states_per_group": S.value, "persistent": bool(pers.value), "workgroups": wg.value,
                "work_items": items.value, "lds_batch": lb.value}

    # ------------------------------------------------- counterfactual utility
    def _utility_args(self, scene, camera, contexts, context_group, group_pl):
        self._codes(contexts, scene)
        _check_tensor(context_group, "context_group", torch.int32, self.device)
        _check_tensor(group_pl, "group_pl", torch.int16, self.device)
        if context_group.shape != (contexts.shape[0],) or group_pl.dim() != 1 or group_pl.shape[0] < 1:
            raise ValueError("context_group must be [J] and group_pl [G] with G >= 1")

    def _ensure_uws(self, scene, camera, G, J, capacity):
        nbytes = _abi.lib().dgs_utility_workspace_bytes(scene.num_packets, ctypes.byref(_c_camera(camera)),
                                                        ctypes.byref(self.tuning), int(G), int(J), int(capacity))
        if nbytes == 0:
            raise ValueError("invalid arguments for dgs_utility_workspace_bytes")
        if getattr(self, "uws", None) is None or self.uws.numel() < nbytes:
            self.uws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        return int(nbytes)

    def utility_items(self, scene: GaussianScene, camera: Camera, contexts: torch.Tensor,
                      context_group: torch.Tensor, group_pl: torch.Tensor, basis) -> int:
        """Work items ``utility`` needs (synchronises; uses the last ``bin``)."""
        _refuse_capture("Renderer.utility_items")
        self._utility_args(scene, camera, contexts, context_group, group_pl)
        G, J = int(group_pl.shape[0]), int(contexts.shape[0])
        nbytes = self._ensure_uws(scene, camera, G, J, 0)
        items = ctypes.c_int64(0)
        _abi.check(_abi.lib().dgs_utility_count(
            ctypes.byref(_c_scene(scene)), ctypes.byref(_c_camera(camera)),
            ctypes.byref(_c_states(contexts, basis, (0, 0, 0))), ctypes.byref(self.tuning), _ptr(self.ws),
            self.ws_bytes, self.capacity, _ptr(context_group), _ptr(group_pl), G, _ptr(self.uws), nbytes,
            ctypes.byref(items), self._stream()))
        return int(items.value)

    def utility(self, scene: GaussianScene, camera: Camera, contexts: torch.Tensor, context_group: torch.Tensor,
                group_pl: torch.Tensor, basis, reference: torch.Tensor, background=(0, 0, 0), lam: float = 0.20,
                item_capacity: Optional[int] = None, out=None) -> torch.Tensor:
        """Eq. (3): Delta_g(m) [J] for contexts [J, P] (u8), each paired with
        group ``group_pl[context_group[j]]`` = (packet << 2) | layer, against
        ``reference`` [H, Wd, 3], from the lists of the last ``bin``.  Without
        ``item_capacity`` the work items are counted first (synchronises)."""
        self._utility_args(scene, camera, contexts, context_group, group_pl)
        _check_tensor(reference, "reference", torch.float32, self.device)
        G, J = int(group_pl.shape[0]), int(contexts.shape[0])
        if item_capacity is None:
            item_capacity = self.utility_items(scene, camera, contexts, context_group, group_pl, basis)
        nbytes = self._ensure_uws(scene, camera, G, J, item_capacity)
        delta = out if out is not None else torch.empty(J, dtype=torch.float32, device=self.device)
        _abi.check(_abi.lib().dgs_utility(
            ctypes.byref(_c_scene(scene)), ctypes.byref(_c_camera(camera)),
            ctypes.byref(_c_states(contexts, basis, background)), ctypes.byref(self.tuning), _ptr(self.ws),
            self.ws_bytes, self.capacity, _ptr(context_group), _ptr(group_pl), G, _ptr(reference), float(lam),
            _ptr(self.uws), nbytes, int(item_capacity), _ptr(delta), self._stream()))
        self.utility_capacity = int(item_capacity)
        return delta

    def utility_check(self) -> int:
        """Synchronise; work items of the last ``utility``; raises DgsError on
        an invalid group or context or an item overflow."""
        _refuse_capture("Renderer.utility_check")
        items = ctypes.c_int64(0)
        _abi.check(_abi.lib().dgs_utility_check(_ptr(self.uws), self.uws.numel(), self.utility_capacity,
                                                ctypes.byref(items), self._stream()))
        return int(items.value)

    def render_psnr(self, scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis,
                    reference: torch.Tensor, background=(0, 0, 0), out=None):
        """PSNR [W] of each state against ``reference`` [H, Wd, 3]."""
        self._codes(codes, scene)
        _check_tensor(reference, "reference", torch.float32, self.device)
        W = int(codes.shape[0])
        self._need_plan(scene, camera, basis, W)
        ps = out if out is not None else torch.empty((W,), dtype=torch.float32, device=self.device)
        _abi.check(_abi.lib().dgs_render_psnr(
            ctypes.byref(_c_scene(scene)), ctypes.byref(_c_camera(camera)),
            ctypes.byref(_c_states(codes, basis, background)), ctypes.byref(self.tuning), _ptr(self.ws),
            self.ws_bytes, self.capacity, _ptr(reference), _ptr(ps), self._stream()))
        self.generation += 1
        return ps

    def backward(self, scene: GaussianScene, camera: Camera, codes, basis, background, image, grad_image,
                 params=None):
        """Parameter gradients (dict of tensors) for dL/d image; the workspace
        must still hold this render's lists (see ``RenderFunction``).  With
        refinement levels the dict also holds ``refine``."""
        p = params or {k: getattr(scene, k) for k in PARAMS}
        grads = {k: torch.empty_like(p[k]) for k in PARAMS}
        if scene.refine is not None:
            grads["refine"] = torch.empty_like(scene.refine)
        g = _abi.SceneGrad(*[_ptr(grads[k]) for k in PARAMS], _ptr(grads.get("refine")))
        image = image.contiguous()
        grad_image = grad_image.contiguous()
        _abi.check(_abi.lib().dgs_backward(
            ctypes.byref(_c_scene(scene, p)), ctypes.byref(_c_camera(camera)),
            ctypes.byref(_c_states(codes, basis, background)), ctypes.byref(self.tuning), _ptr(self.ws),
            self.ws_bytes, self.capacity, _ptr(image), _ptr(grad_image), ctypes.byref(g), self._stream()))
        return grads


class RenderFunction(torch.autograd.Function):
    """Differentiable batched render: gradients for the six parameter tensors
    (and the refinement levels, passed as a seventh tensor, when the scene has
    them).

    The backward replays each tile's compositing from the forward's sorted
    lists.  If the renderer's workspace was reused by another call in between,
    the lists are rebuilt first (one extra forward)."""

    @staticmethod
    def forward(ctx, renderer, scene, camera, codes, basis, background, *params):
        p = dict(zip(PARAMS, params))
        if len(params) > len(PARAMS):
            scene = scene.with_params(refine=params[len(PARAMS)])
        img = renderer.render(scene, camera, codes, basis, background, params=p)
        ctx.renderer, ctx.scene, ctx.camera = renderer, scene, camera
        ctx.codes, ctx.basis, ctx.background = codes, basis, background
        ctx.generation = renderer.generation
        ctx.save_for_backward(img, *params)
        return img

    @staticmethod
    def backward(ctx, grad_image):
        img, *params = ctx.saved_tensors
        p = dict(zip(PARAMS, params))
        r = ctx.renderer
        if r.generation != ctx.generation:
            # another call reused the workspace between this forward and its
            # backward; rebuilding the lists is a render of its own, which a
            # captured training step must not hide inside its backward
            _refuse_capture("a re-render in RenderFunction.backward (the workspace was reused after the forward)")
            r.render(ctx.scene, ctx.camera, ctx.codes, ctx.basis, ctx.background, params=p)
        g = r.backward(ctx.scene, ctx.camera, ctx.codes, ctx.basis, ctx.background, img, grad_image, params=p)
        out = tuple(g[k] for k in PARAMS) + ((g["refine"],) if len(params) > len(PARAMS) else ())
        return (None, None, None, None, None, None) + out


def distortion(images: torch.Tensor, reference: torch.Tensor, lam: float = 0.20) -> torch.Tensor:
    """D = MSE + lam (1 - SSIM) of each image [W, H, Wd, 3] against
    ``reference`` [H, Wd, 3] (Sec. 4's distortion), computed on the device."""
    _check_tensor(images, "images", torch.float32, images.device)
    _check_tensor(reference, "reference", torch.float32, images.device)
    if images.dim() != 4 or images.shape[-1] != 3 or tuple(reference.shape) != tuple(images.shape[1:]):
        raise ValueError("images must be [W, H, Wd, 3] and reference [H, Wd, 3]")
    W, H, Wd = (int(x) for x in images.shape[:3])
    L = _abi.lib()
    nbytes = L.dgs_distortion_scratch_bytes(W, Wd, H)
    scratch = torch.empty(max(int(nbytes), 8), dtype=torch.uint8, device=images.device)
    d = torch.empty(W, dtype=torch.float32, device=images.device)
    with torch.cuda.device(images.device):
        st = ctypes.c_void_p(torch.cuda.current_stream(images.device).cuda_stream)
        _abi.check(L.dgs_distortion(_ptr(images), W, Wd, H, _ptr(reference), float(lam), _ptr(scratch),
                                    int(nbytes), _ptr(d), st))
    return d


def risk_adjusted(values: torch.Tensor, offsets: torch.Tensor, alpha: float = 0.25, beta: float = 0.05,
                  quantile: float = 0.10) -> torch.Tensor:
    """Eq. (4) per group: [G, 4] = (mean, quantile, std, risk-adjusted) of
    values[offsets[k]:offsets[k+1]] (float32 / int32 device tensors)."""
    _check_tensor(values, "values", torch.float32, values.device)
    _check_tensor(offsets, "offsets", torch.int32, values.device)
    G = int(offsets.shape[0]) - 1
    out = torch.empty((max(G, 0), 4), dtype=torch.float32, device=values.device)
    with torch.cuda.device(values.device):
        st = ctypes.c_void_p(torch.cuda.current_stream(values.device).cuda_stream)
        _abi.check(_abi.lib().dgs_risk_adjusted(_ptr(values), _ptr(offsets), G, float(alpha), float(beta),
                                                float(quantile), _ptr(out), st))
    return out


CHANNEL_DTYPE = np.dtype([("p_gb", np.float32), ("p_bg", np.float32), ("loss_good", np.float32),
                          ("loss_bad", np.float32), ("p_start_bad", np.float32), ("deadline", np.int32)])


def channels_to_device(channels, device) -> torch.Tensor:
    """A structured array of CHANNEL_DTYPE (one dgs_channel per world) as
    device bytes [W, 24] for ``sample_states``."""
    a = np.ascontiguousarray(channels, dtype=CHANNEL_DTYPE)
    return torch.from_numpy(a.view(np.uint8).reshape(a.shape[0], CHANNEL_DTYPE.itemsize).copy()).to(device)


def sample_states(channels: torch.Tensor, num_packets: int, num_layers: int, seed: int, out=None) -> torch.Tensor:
    """Delivery codes [W, num_packets] (uint8) drawn on the device from one
    Gilbert-Elliott / deadline channel per world (``channels``: uint8 [W, 24]
    from ``channels_to_device``)."""
    if channels.dtype != torch.uint8 or channels.dim() != 2 or channels.shape[1] != CHANNEL_DTYPE.itemsize:
        raise ValueError("channels must be uint8 [W, 24] (see channels_to_device)")
    if not channels.is_contiguous():
        raise ValueError("channels must be contiguous")
    W = int(channels.shape[0])
    codes = out if out is not None else torch.empty((W, int(num_packets)), dtype=torch.uint8, device=channels.device)
    with torch.cuda.device(channels.device):
        st = ctypes.c_void_p(torch.cuda.current_stream(channels.device).cuda_stream)
        _abi.check(_abi.lib().dgs_sample_states(_ptr(channels), W, int(num_packets), int(num_layers),
                                                ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), _ptr(codes), st))
    return codes


# Eq. (2) weights the paper locks (Sec. 4)
OBJECTIVE_WEIGHTS = dict(lambda_ssim=0.20, lambda_c=0.30, alpha=0.05, lambda_t=0.10, lambda_m=2.0, lambda_a=0.50)


def _index_tensor(x, name, device, pairs=False):
    if x is None:
        return None, 0
    t = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x, np.int32).reshape(-1))
    t = t.to(device=device, dtype=torch.int32).contiguous().reshape(-1)
    if pairs and t.numel() % 2:
        raise ValueError(f"{name} must hold (a, b) pairs")
    return t, int(t.numel() // (2 if pairs else 1))


class Objective:
    """Eq. (2) of a training batch on the device: ``__call__`` returns
    (loss parts [6] = L, E, CVaR, F, M, anchor; D per image; dL/d images).
    Keeps its scratch buffer between calls."""

    def __init__(self, device, weights=None):
        self.device = torch.device(device)
        w = dict(OBJECTIVE_WEIGHTS)
        w.update(weights or {})
        self.weights = _abi.ObjectiveWeights(*(float(w[k]) for k in ("lambda_ssim", "lambda_c", "alpha",
                                                                         "lambda_t", "lambda_m", "lambda_a")))
        self.scratch = None
        self.scratch_bytes = 0

    def __call__(self, images, targets, target_of, expect, anchor=None, mono=None, temporal=None, grad=True,
                 out_grad=None):
        dev = self.device
        _check_tensor(images, "images", torch.float32, dev)
        _check_tensor(targets, "targets", torch.float32, dev)
        if images.dim() != 4 or images.shape[-1] != 3 or targets.dim() != 4 or \
                tuple(targets.shape[1:]) != tuple(images.shape[1:]):
            raise ValueError("images [K, H, W, 3] and targets [T, H, W, 3] of one image size")
        K, H, Wd = (int(x) for x in images.shape[:3])
        tof, nt = _index_tensor(target_of, "target_of", dev)
        if nt != K:
            raise ValueError("target_of needs one entry per image")
        ex, ne = _index_tensor(expect, "expect", dev)
        an, na = _index_tensor(anchor, "anchor", dev)
        mo, nm = _index_tensor(mono, "mono", dev, pairs=True)
        te, nq = _index_tensor(temporal, "temporal", dev, pairs=True)
        L = _abi.lib()
        nbytes = int(L.dgs_objective_scratch_bytes(K, Wd, H, nq))
        if nbytes == 0:
            raise ValueError("invalid sizes for dgs_objective")
        if nbytes > self.scratch_bytes:
            self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            self.scratch_bytes = nbytes
        loss = torch.empty(6, dtype=torch.float32, device=dev)
        d = torch.empty(K, dtype=torch.float32, device=dev)
        g = None
        if grad:
            g = out_grad if out_grad is not None else torch.empty_like(images)
        with torch.cuda.device(dev):
            st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
            _abi.check(L.dgs_objective(_ptr(images), K, Wd, H, _ptr(targets), int(targets.shape[0]), _ptr(tof),
                                       _ptr(ex), ne, _ptr(an), na, _ptr(mo), nm, _ptr(te), nq,
                                       ctypes.byref(self.weights), _ptr(loss), _ptr(d), _ptr(g),
                                       _ptr(self.scratch), self.scratch_bytes, st))
        return loss, d, g

    def check(self):
        """Synchronise; raises DgsError if the last call met an index out of range."""
        _refuse_capture("Objective.check")
        with torch.cuda.device(self.device):
            st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            _abi.check(_abi.lib().dgs_objective_check(_ptr(self.scratch), self.scratch_bytes, st))


class ObjectiveFunction(torch.autograd.Function):
    """Eq. (2) as a differentiable function of the rendered images: the
    forward returns L, the backward the device gradient scaled by dL."""

    @staticmethod
    def forward(ctx, objective, images, targets, target_of, expect, anchor, mono, temporal):
        loss, d, g = objective(images.detach().contiguous(), targets, target_of, expect, anchor, mono, temporal)
        ctx.image_grad = g
        return loss[0].clone()

    @staticmethod
    def backward(ctx, grad_loss):
        return (None, ctx.image_grad * grad_loss, None, None, None, None, None, None)


class L1Loss:
    """Mean absolute error of images [K, H, W, 3] against targets [T, H, W, 3]
    (image k against ``targets[target_of[k]]``, default all target 0) on the
    device; keeps its scratch buffer between calls.  ``loss`` returns the
    scalar, ``grad`` dL/d images scaled by ``dloss`` (a device scalar or
    None for 1)."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.scratch = None
        self.scratch_bytes = 0

    def _args(self, images, targets, target_of):
        dev = self.device
        _check_tensor(images, "images", torch.float32, dev)
        _check_tensor(targets, "targets", torch.float32, dev)
        if images.dim() != 4 or images.shape[-1] != 3 or targets.dim() != 4 or \
                tuple(targets.shape[1:]) != tuple(images.shape[1:]):
            raise ValueError("images [K, H, W, 3] and targets [T, H, W, 3] of one image size")
        K, H, Wd = (int(x) for x in images.shape[:3])
        tof = None
        if target_of is not None:
            tof, nt = _index_tensor(target_of, "target_of", dev)
            if nt != K:
                raise ValueError("target_of needs one entry per image")
        return K, H, Wd, tof

    def loss(self, images, targets, target_of=None):
        K, H, Wd, tof = self._args(images, targets, target_of)
        L = _abi.lib()
        nbytes = int(L.dgs_l1_scratch_bytes(K, Wd, H))
        if nbytes == 0:
            raise ValueError("invalid sizes for dgs_l1_loss")
        if nbytes > self.scratch_bytes:
            self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.scratch_bytes = nbytes
        out = torch.empty((), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            _abi.check(L.dgs_l1_loss(_ptr(images), K, Wd, H, _ptr(targets), int(targets.shape[0]), _ptr(tof),
                                     _ptr(out), _ptr(self.scratch), self.scratch_bytes, st))
        return out

    def grad(self, images, targets, target_of=None, dloss=None):
        K, H, Wd, tof = self._args(images, targets, target_of)
        if dloss is not None:
            _check_tensor(dloss, "dloss", torch.float32, self.device)
            if dloss.numel() != 1:
                raise ValueError("dloss must hold one value")
        g = torch.empty_like(images)
        with torch.cuda.device(self.device):
            st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            _abi.check(_abi.lib().dgs_l1_loss_grad(_ptr(images), K, Wd, H, _ptr(targets), int(targets.shape[0]),
                                                   _ptr(tof), _ptr(dloss), _ptr(g), st))
        return g

    def check(self):
        """Synchronise; raises DgsError if the last loss met a target index out of range."""
        _refuse_capture("L1Loss.check")
        with torch.cuda.device(self.device):
            st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            _abi.check(_abi.lib().dgs_objective_check(_ptr(self.scratch), self.scratch_bytes, st))


class L1Function(torch.autograd.Function):
    """The L1 loss as a differentiable function of the images: one device
    pass for the loss, one for the gradient (scaled by the upstream
    gradient on the device, no host synchronisation)."""

    @staticmethod
    def forward(ctx, l1, images, targets, target_of):
        x = images.detach().contiguous()
        ctx.l1, ctx.target_of = l1, target_of
        ctx.save_for_backward(x, targets)
        return l1.loss(x, targets, target_of)

    @staticmethod
    def backward(ctx, grad_loss):
        x, targets = ctx.saved_tensors
        dl = grad_loss.detach().to(torch.float32).contiguous().reshape(1)
        return None, ctx.l1.grad(x, targets, ctx.target_of, dl), None, None


def l1_loss(images, targets, target_of=None, l1: Optional[L1Loss] = None):
    """Differentiable mean |images - targets[target_of]| on the device."""
    return L1Function.apply(l1 if l1 is not None else L1Loss(images.device), images, targets, target_of)


def render(renderer: Renderer, scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis,
           background=(0, 0, 0)):
    """Differentiable render of every state in ``codes`` -> [W, H, Wd, 3]
    (gradients also reach ``scene.refine`` when the scene has levels)."""
    params = [getattr(scene, k) for k in PARAMS]
    if scene.refine is not None:
        params.append(scene.refine)
    return RenderFunction.apply(renderer, scene, camera, codes, tuple(float(b) for b in basis),
                                tuple(float(x) for x in background), *params)


class StreamPipeline:
    """Successive renders overlapped on ``depth`` streams.

    Call ``i`` runs the whole path (``bin``, then ``composite``) on stream
    ``i % depth`` with a renderer, hence a workspace, of its own.  Calls in
    flight share no device memory apart from their read-only inputs, so the
    binning of one call (a chain of short launches that leave most of the
    chip idle) and the last workgroups of its compositing run beside the
    compositing of the calls before it.  Every call is the full path: the
    images equal ``Renderer.render``'s bit for bit.

    Each call first waits for the work the caller has queued on its current
    stream.  The results are ready on the caller's stream after ``join()``;
    until then a call's inputs must not change and its image (a caller's
    ``out`` buffer included) must not be read or freed.  The streams have the
    default priority."""

    def __init__(self, device="cuda", depth: int = 3, **renderer_kwargs):
        if int(depth) < 1:
            raise ValueError(f"depth must be at least 1, got {depth}")
        self.depth = int(depth)
        self.renderers = [Renderer(device, **renderer_kwargs) for _ in range(self.depth)]
        self.device = self.renderers[0].device
        self.streams = [torch.cuda.Stream(self.device) for _ in range(self.depth)]
        self.calls = 0

    def plan(self, scene: GaussianScene, camera: Camera, basis, max_states: int) -> int:
        """Plan every renderer (synchronises); returns the instance count."""
        return [r.plan(scene, camera, basis, max_states) for r in self.renderers][0]

    def render(self, scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis, background=(0, 0, 0),
               out=None) -> torch.Tensor:
        """Images [W, H, Wd, 3] of every state in ``codes``, queued on the next stream."""
        j = self.calls % self.depth
        self.calls += 1
        cur = torch.cuda.current_stream(self.device)
        s = self.streams[j]
        s.wait_stream(cur)
        r = self.renderers[j]
        with torch.cuda.stream(s):
            r._need_plan(scene, camera, basis, int(codes.shape[0]))
            r.bin(scene, camera, basis)
            img = r.composite(scene, camera, codes, basis, background, out=out)
        if out is None:
            img.record_stream(cur)  # allocated on s, read later on the caller's stream
        return img

    def join(self):
        """Make the caller's current stream wait for every call so far."""
        cur = torch.cuda.current_stream(self.device)
        for s in self.streams:
            cur.wait_stream(s)

    def check(self) -> int:
        """Wait for every call so far (``join()``), synchronise, and raise
        DgsError if any renderer's last binning overflowed; returns the
        largest instance count."""
        self.join()
        return max(r.check() for r in self.renderers)


class CapturedRender:
    """``bin`` + ``composite`` (or ``composite_psnr``) of fixed tensors captured
    in one HIP graph; ``replay()`` relaunches the whole path with one call.

    The scene, codes and reference tensors are read at every replay, so their
    contents may change between replays (not their shapes or addresses).  The
    graph holds the renderer's workspace (kept alive here); until ``close()``
    the renderer refuses to plan again or to replace that workspace."""

    def __init__(self, renderer: Renderer, scene: GaussianScene, camera: Camera, codes: torch.Tensor, basis,
                 background=(0, 0, 0), reference: Optional[torch.Tensor] = None):
        r = renderer
        W = int(codes.shape[0])
        r._need_plan(scene, camera, basis, W)
        dev = r.device
        if reference is None:
            self.out = torch.empty((W, camera.height, camera.width, 3), dtype=torch.float32, device=dev)
        else:
            self.out = torch.empty((W,), dtype=torch.float32, device=dev)

        def body():
            r.bin(scene, camera, basis)
            if reference is None:
                r.composite(scene, camera, codes, basis, background, out=self.out)
            else:
                r.composite_psnr(scene, camera, codes, basis, reference, background, out=self.out)

        side = torch.cuda.Stream(dev)  # default priority
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            body()
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            body()
        self.renderer = r
        # the graph's kernels hold raw pointers into these tensors
        self._keep = (scene, codes, reference, r.ws, r.uws)
        r.live_captures += 1
        self._closed = False

    def replay(self) -> torch.Tensor:
        if self._closed:
            raise RuntimeError("this CapturedRender was closed")
        self.graph.replay()
        return self.out

    def close(self):
        """Release the graph and let the renderer plan again."""
        if not self._closed:
            self._closed = True
            self.graph.reset()
            self._keep = None
            self.renderer.live_captures -= 1

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass
