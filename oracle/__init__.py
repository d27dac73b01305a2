"""Reference (oracle) renderer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the bench's CPU-baseline leg
may import this package.  The renderer library and its Python binding never
import, load or call anything here, and this package imports nothing from
them.

Contents:
* ``liboracle.so`` (``oracle.c``): FP64 per-pixel renderer, FP64 geometry,
  FP32 mirror of the integer decisions (culling, tile rectangles, depth keys).
* ``tile_lists``: per-tile (depth, index) order via ``numpy.lexsort``.
* ``refined_scene`` / ``render_refined``: attribute-level prefix refinement
  (Sec. 3): every delivery state decodes to a plain scene, rendered as above.
* ``grad``: FP64 dense formulation in plain PyTorch CPU ops whose autograd
  gives the exact derivative with every discrete decision frozen.
"""

from __future__ import annotations

import copy
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

# field order of or_geometry_f64's output rows
GEOM_FIELDS = ("u", "v", "a", "b", "c", "conA", "conB", "conC", "o", "r", "g", "b_", "X", "Y", "Z")

_lib = None


class _Scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("rank", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("num_packets", ctypes.c_int32), ("num_contexts", ctypes.c_int32),
                ("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p),
                ("color", ctypes.c_void_p), ("temporal", ctypes.c_void_p),
                ("packet_layer", ctypes.c_void_p), ("cluster_affine", ctypes.c_void_p),
                ("offset", ctypes.c_void_p)]


class _Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("near_z", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "oracle.c")
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.or_exp_f32.restype = ctypes.c_float
        L.or_exp_f32.argtypes = [ctypes.c_float]
        L.or_mirror_f32.restype = ctypes.c_int
        L.or_geometry_f64.restype = ctypes.c_int
        L.or_render.restype = ctypes.c_int
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class _Pinned:
    """Keeps the numpy arrays referenced by a ctypes struct alive."""

    def __init__(self, scene, cam):
        self.arrs = dict(mean=_f32(scene.mean), log_scale=_f32(scene.log_scale),
                         quat=_f32(scene.quat), opacity_logit=_f32(scene.opacity_logit),
                         color=_f32(scene.color), temporal=_f32(scene.temporal),
                         packet_layer=np.ascontiguousarray(scene.packet_layer, dtype=np.uint16))
        aff = None
        if scene.cluster_affine is not None:
            aff = _f32(scene.cluster_affine)
            self.arrs["cluster_affine"] = aff
        off = getattr(scene, "offset", None)
        if off is not None:
            self.arrs["offset"] = _f32(off)
        ptr = lambda k: self.arrs[k].ctypes.data if k in self.arrs else None  # noqa: E731
        n = scene.mean.shape[1]
        self.scene = _Scene(n, scene.rank, scene.sh_degree, scene.num_clusters * scene.num_contexts,
                            scene.num_contexts, ptr("mean"), ptr("log_scale"), ptr("quat"),
                            ptr("opacity_logit"), ptr("color"), ptr("temporal"),
                            ptr("packet_layer"), ptr("cluster_affine"), ptr("offset"))
        c = _Camera()
        R = _f32(cam.R_cw).reshape(9)
        t = _f32(cam.t_cw).reshape(3)
        for k in range(9):
            c.R[k] = float(R[k])
        for k in range(3):
            c.t[k] = float(t[k])
        c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
        c.near_z = cam.near
        c.width, c.height = cam.width, cam.height
        self.cam = c


def exp_f32(x: float) -> np.float32:
    return np.float32(lib().or_exp_f32(ctypes.c_float(x)))


def geometry_f64(scene, cam, basis) -> dict:
    """Per-Gaussian FP64 projection: dict of [N] float64 arrays (GEOM_FIELDS)."""
    pin = _Pinned(scene, cam)
    n = scene.mean.shape[1]
    out = np.zeros((len(GEOM_FIELDS), max(n, 1)), dtype=np.float64)
    b = _f32(basis) if len(basis) else np.zeros(1, np.float32)
    rc = lib().or_geometry_f64(ctypes.byref(pin.scene), ctypes.byref(pin.cam),
                               b.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    return {k: out[j, :n] for j, k in enumerate(GEOM_FIELDS)}


def mirror_f32(scene, cam, basis, tile_w: int = 16, tile_h: int = 16) -> dict:
    """FP32 integer decisions: depth z32 (+ its uint32 bits), u, v, a, b, c,
    the conic scaled for the base-2 exponent (cA, cB, cC: q' = cA dx^2 +
    cB dx dy + cC dy^2), tile rectangle [x0, y0, x1, y1) and validity."""
    pin = _Pinned(scene, cam)
    n = scene.mean.shape[1]
    f = np.zeros((9, max(n, 1)), dtype=np.float32)
    r = np.zeros((4, max(n, 1)), dtype=np.int32)
    v = np.zeros(max(n, 1), dtype=np.int32)
    b = _f32(basis) if len(basis) else np.zeros(1, np.float32)
    rc = lib().or_mirror_f32(ctypes.byref(pin.scene), ctypes.byref(pin.cam),
                             b.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(tile_w),
                             ctypes.c_int(tile_h), f.ctypes.data_as(ctypes.c_void_p),
                             r.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError("tile sizes must be powers of two")
    z32 = f[0, :n].copy()
    return dict(z32=z32, zbits=z32.view(np.uint32), u=f[1, :n].copy(), v=f[2, :n].copy(),
                a=f[3, :n].copy(), b=f[4, :n].copy(), c=f[5, :n].copy(),
                cA=f[6, :n].copy(), cB=f[7, :n].copy(), cC=f[8, :n].copy(), rect=r[:, :n].copy(), valid=v[:n].astype(bool), tile_w=tile_w, tile_h=tile_h)


def tile_lists(mirror: dict, width: int, height: int, present=None):
    """Per-tile Gaussian lists in the order (tile id, depth bits, index).

    Returns (ranges [tiles][2] int64 half-open into ids, ids [M] int64,
    keys [M] uint64 = tile << 32 | depth bits).  ``present`` (bool [N])
    restricts the lists to a subset.  The order is numpy.lexsort's, i.e. a
    stable sort on the three keys."""
    tw, th = mirror["tile_w"], mirror["tile_h"]
    tiles_x = (width + tw - 1) // tw
    tiles_y = (height + th - 1) // th
    rect = mirror["rect"].astype(np.int64)
    ok = mirror["valid"].copy()
    if present is not None:
        ok &= present
    nx = np.clip(rect[2] - rect[0], 0, None)
    ny = np.clip(rect[3] - rect[1], 0, None)
    cnt = np.where(ok, nx * ny, 0)
    total = int(cnt.sum())
    ids = np.repeat(np.arange(cnt.size, dtype=np.int64), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    k = np.arange(total, dtype=np.int64) - start
    nxr = np.repeat(np.maximum(nx, 1), cnt)
    tx = np.repeat(rect[0], cnt) + k % nxr
    ty = np.repeat(rect[1], cnt) + k // nxr
    tile = ty * tiles_x + tx
    zb = mirror["zbits"].astype(np.int64)[ids]
    order = np.lexsort((ids, zb, tile))
    tile, ids, zb = tile[order], ids[order], zb[order]
    counts = np.bincount(tile, minlength=tiles_x * tiles_y)
    ends = np.cumsum(counts)
    ranges = np.stack([ends - counts, ends], axis=1)
    keys = (tile.astype(np.uint64) << np.uint64(32)) | zb.astype(np.uint64)
    return ranges, ids, keys


def render(scene, cam, basis, codes, background, pixels=None) -> dict:
    """FP64 render.  ``pixels``: None (all, row-major) or int array [K][2] of
    (x, y).  Returns image [W][K][3] (or [W][H][Wd][3] when pixels is None),
    tfinal, budget, ncomp with matching leading shapes."""
    pin = _Pinned(scene, cam)
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    W = codes.shape[0]
    assert codes.shape[1] == scene.num_clusters * scene.num_contexts
    if pixels is None:
        npix = cam.width * cam.height
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        npix = pix.shape[0]
    image = np.zeros((W, npix, 3), dtype=np.float64)
    tfinal = np.zeros((W, npix), dtype=np.float64)
    budget = np.zeros((W, npix), dtype=np.float64)
    ncomp = np.zeros((W, npix), dtype=np.int32)
    bg = _f32(background)
    b = _f32(basis) if len(basis) else np.zeros(1, np.float32)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = lib().or_render(ctypes.byref(pin.scene), ctypes.byref(pin.cam), vp(b), ctypes.c_int(W),
                         vp(codes), vp(bg), ctypes.c_int64(npix),
                         vp(pix) if pix is not None else None, vp(image), vp(tfinal), vp(budget),
                         vp(ncomp))
    if rc != 0:
        raise MemoryError("oracle render failed")
    if pixels is None:
        H, Wd = cam.height, cam.width
        return dict(image=image.reshape(W, H, Wd, 3), tfinal=tfinal.reshape(W, H, Wd),
                    budget=budget.reshape(W, H, Wd), ncomp=ncomp.reshape(W, H, Wd))
    return dict(image=image, tfinal=tfinal, budget=budget, ncomp=ncomp)


def psnr(image, reference) -> np.ndarray:
    """PSNR per state with peak 1: 10 log10(1 / max(MSE, 1e-10)), MSE over
    every pixel and channel."""
    d = np.asarray(image, np.float64) - np.asarray(reference, np.float64)[None]
    mse = (d * d).reshape(d.shape[0], -1).mean(axis=1)
    return 10.0 * np.log10(1.0 / np.maximum(mse, 1e-10))


def present_mask(scene, codes_row) -> np.ndarray:
    """bool [N]: Gaussian present under one state's codes (layer < code)."""
    pl = scene.packet_layer.astype(np.int64)
    return (pl & 3) < np.asarray(codes_row, np.int64)[pl >> 2]


# ------------------------------------------------- attribute refinement levels
def refine_rows(sh_degree: int) -> int:
    """Rows of one refinement level: position residual 3, log-scale 3,
    quaternion 4, opacity logit 1, colour 3 (RGB) or 12 (SH-1)."""
    return 11 + (3 if sh_degree == 0 else 12)


def refined_scene(scene, refine, codes_row):
    """The plain scene that one delivery state decodes to (Sec. 3: scale,
    rotation, opacity and colour are a base plus three refinements; the
    position carries residual levels on top of Eq. (1)'s deformation).

    ``refine``: float32 [3][rows][N], level j = 1..3 at index j - 1, rows as
    in ``refine_rows``.  A Gaussian whose packet is delivered to depth d
    (code d + 1, codes above 4 act as 4) takes base + level 1 + ... + level
    d, summed in FP32 in that order (the storage precision of every
    attribute); its position residual o = level 1 + ... + level d (0 at d = 0)
    is added after the deformation.  Presence is unchanged: layer < code."""
    refine = np.asarray(refine, np.float32)
    n = scene.mean.shape[1]
    rows = refine_rows(scene.sh_degree)
    assert refine.shape == (3, rows, n), (refine.shape, (3, rows, n))
    pl = scene.packet_layer.astype(np.int64)
    depth = np.minimum(np.asarray(codes_row, np.int64)[pl >> 2], 4) - 1  # -1: packet absent
    base = np.concatenate([np.zeros((3, n), np.float32), _f32(scene.log_scale), _f32(scene.quat),
                           _f32(scene.opacity_logit).reshape(1, n), _f32(scene.color)])
    acc = base.copy()
    for j in range(1, 4):
        take = depth >= j
        acc[:, take] = acc[:, take] + refine[j - 1][:, take]
    out = copy.copy(scene)
    out.offset = np.ascontiguousarray(acc[:3])
    out.log_scale = np.ascontiguousarray(acc[3:6])
    out.quat = np.ascontiguousarray(acc[6:10])
    out.opacity_logit = np.ascontiguousarray(acc[10])
    out.color = np.ascontiguousarray(acc[11:])
    return out


def render_refined(scene, refine, cam, basis, codes, background, pixels=None) -> dict:
    """FP64 render of a scene with refinement levels: each state's plain
    scene (``refined_scene``) through ``render``.  Same outputs as ``render``."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    parts = [render(refined_scene(scene, refine, codes[w]), cam, basis, codes[w:w + 1], background, pixels)
             for w in range(codes.shape[0])]
    if not parts:
        return render(scene, cam, basis, codes, background, pixels)
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


# ----------------------------------------------------------- state sampler
class _Channel(ctypes.Structure):
    _fields_ = [("p_gb", ctypes.c_float), ("p_bg", ctypes.c_float), ("loss_good", ctypes.c_float),
                ("loss_bad", ctypes.c_float), ("p_start_bad", ctypes.c_float), ("deadline", ctypes.c_int32)]


CHANNEL_DTYPE = np.dtype([("p_gb", np.float32), ("p_bg", np.float32), ("loss_good", np.float32),
                          ("loss_bad", np.float32), ("p_start_bad", np.float32), ("deadline", np.int32)])


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter under a 2-word key."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(c.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                           out.ctypes.data_as(ctypes.c_void_p))
    return out


def sample_states(channels: np.ndarray, num_packets: int, num_layers: int, seed: int) -> np.ndarray:
    """Delivery codes [W][P] of the Gilbert-Elliott / deadline sampler
    (``channels``: structured array of CHANNEL_DTYPE, one per world)."""
    ch = np.ascontiguousarray(channels, dtype=CHANNEL_DTYPE)
    W = ch.shape[0]
    codes = np.zeros((W, num_packets), dtype=np.uint8)
    rc = lib().or_sample_states(ch.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(W), ctypes.c_int(num_packets),
                                ctypes.c_int(num_layers), ctypes.c_uint64(seed),
                                codes.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    return codes

