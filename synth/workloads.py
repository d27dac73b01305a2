"""Synthetic dynamic Gaussian scenes, cameras and delivery-state codes.

Every array is drawn from ``numpy.random.default_rng(SeedSequence([2606,
workload_index, stream]))`` with stream 0 = scene, 1 = delivery states,
2 = parameter perturbation, 3 = finite-difference subscene, 4 = refinement
levels, 5 = cluster affines.  Values are drawn in
float64 and stored as float32; both the oracle and the GPU path read the
float32 values.

Layouts (component-major structure of arrays, ``[k][N]``):

* ``mean [3][N]``        canonical means (the paper's mu-bar in Eq. (1), Sec. 3)
* ``log_scale [3][N]``   per-axis log standard deviations
* ``quat [4][N]``        rotation quaternion (w, x, y, z)
* ``opacity_logit [N]``
* ``color [3][N]`` (RGB) or ``[12][N]`` (degree-1 spherical harmonics,
  coefficient-major: row index = coef*3 + channel)
* ``temporal [3R][N]``   per-Gaussian temporal coefficients q_{i,r} of Eq. (1),
  row index = r*3 + axis
* ``packet_layer [N]``   uint16 ``(packet << 2) | layer`` with
  ``packet = cluster * K + context``

Refinement levels (optional) are ``refine [3][rows][N]``, level j = 1..3 at
index j - 1, rows: position residual 3, log-scale 3, quaternion 4, opacity
logit 1, colour 3 or 12.  A Gaussian delivered to depth d carries base +
levels 1..d; the position residuals are added after the deformation.

Delivery states are ``codes [W][P]`` uint8: 0 = packet absent, d+1 = prefix
depth d (layers 0..d delivered).  A Gaussian of layer l in packet p is present
in state w iff ``l < codes[w][p]``.  The prefix encoding is dependency-closed
by construction (Sec. 4: dependencies are enforced before masks are formed;
Sec. 3: one base and three refinement groups per cluster).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Optional

import numpy as np


@dataclass
class SceneArrays:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity_logit: np.ndarray
    color: np.ndarray
    temporal: np.ndarray
    packet_layer: np.ndarray
    num_clusters: int
    num_contexts: int
    rank: int
    sh_degree: int
    cluster_affine: Optional[np.ndarray] = None  # [C][12] row-major 3x4, None = identity

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @property
    def num_packets(self) -> int:
        return self.num_clusters * self.num_contexts


@dataclass
class CameraArrays:
    R_cw: np.ndarray  # float32 [3][3], world -> camera rotation (rows: right, down, forward)
    t_cw: np.ndarray  # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.01


@dataclass
class Workload:
    name: str
    index: int
    scene: SceneArrays
    camera: CameraArrays
    codes: np.ndarray  # uint8 [W][P]
    basis: np.ndarray  # float32 [R]
    t: float
    background: np.ndarray  # float32 [3]
    batch: int = 0  # states per launch when the workload is swept in batches (0 = all)
    total_states: int = 0  # states in the full sweep (0 = codes.shape[0])


# name -> recipe.  ``index`` is the workload's seed index.
WORKLOADS = {
    # 4,096 Gaussians, 8 clusters x 4 contexts, 1 layer, 128x128, 16 states.
    "g4k_128px_16states": dict(index=1, n=4096, clusters=8, contexts=4, layers=1,
                               width=128, height=128, states=16, color="rgb",
                               masks=("bernoulli", 0.7, 0.7)),
    # 250,000 Gaussians, 32x32x4 packets/layers, 800x800, 64 states (forward only).
    "g250k_800px_64states": dict(index=2, n=250_000, clusters=32, contexts=32, layers=4,
                                 width=800, height=800, states=64, color="sh1",
                                 masks=("present_depth", 0.3, 1.0)),
    # 2.7M Gaussians, 64x64x4, 1920x1080, 256 states with present fractions 5%..100%.
    "g2700k_1080p_256states": dict(index=3, n=2_700_000, clusters=64, contexts=64, layers=4,
                                   width=1920, height=1080, states=256, color="sh1",
                                   masks=("binomial_ramp", 0.05, 1.0)),
    # 250,000 Gaussians, 1280x720, 8 states; forward + L1 loss + backward.
    "g250k_720p_8states_fwdbwd": dict(index=4, n=250_000, clusters=32, contexts=32, layers=4,
                                      width=1280, height=720, states=8, color="sh1",
                                      masks=("present_depth", 0.3, 1.0)),
    # 1M Gaussians, 64x16, 960x540, 32,768 states swept in batches of 512 (PSNR only).
    "g1m_540p_32768states_psnr": dict(index=5, n=1_000_000, clusters=64, contexts=16, layers=1,
                                      width=960, height=540, states=512, color="sh1",
                                      masks=("bernoulli_uniform", 0.2, 1.0),
                                      batch=512, total_states=32768),
}


def _rng(index: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2606, index, stream]))


def variance_split(points: np.ndarray, num_leaves: int) -> np.ndarray:
    """Deterministic variance split (Sec. 3): recursively halve the point set
    at the median of its largest-variance axis (ties by index) until
    ``num_leaves`` leaves (a power of two) remain; leaves are numbered in
    depth-first order.  ``points`` is (N, 3)."""
    n = points.shape[0]
    if num_leaves & (num_leaves - 1):
        raise ValueError("num_leaves must be a power of two")
    labels = np.zeros(n, dtype=np.int64)
    stack = [(np.arange(n), 0, num_leaves)]
    while stack:
        idx, first, count = stack.pop()
        if count == 1 or idx.size == 0:
            labels[idx] = first
            continue
        pts = points[idx]
        axis = int(np.argmax(pts.var(axis=0))) if idx.size > 1 else 0
        order = np.lexsort((idx, pts[:, axis]))
        srt = idx[order]
        half = srt.size // 2
        stack.append((srt[half:], first + count // 2, count // 2))
        stack.append((srt[:half], first, count // 2))
    return labels


def make_scene(n: int, clusters: int, contexts: int, layers: int, color: str,
               rank: int = 2, index: int = 0, stream: int = 0) -> SceneArrays:
    """Draw a scene: means U[-1,1]^3, log-scales N(-3,0.3), unit quaternions
    from normalised N(0,1)^4, opacity logits N(0,1), RGB U[0,1] or SH-1
    coefficients N(0,0.2), temporal coefficients N(0,0.05), uniform contexts,
    uniform layers 0..layers-1."""
    rng = _rng(index, stream)
    mean = rng.uniform(-1.0, 1.0, size=(n, 3))
    log_scale = rng.normal(-3.0, 0.3, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logit = rng.normal(0.0, 1.0, size=n)
    if color == "rgb":
        col = rng.uniform(0.0, 1.0, size=(n, 3))
        sh_degree = 0
    elif color == "sh1":
        col = rng.normal(0.0, 0.2, size=(n, 12))
        sh_degree = 1
    else:
        raise ValueError(color)
    temporal = rng.normal(0.0, 0.05, size=(n, 3 * rank))
    context = rng.integers(0, contexts, size=n)
    layer = rng.integers(0, layers, size=n) if layers > 1 else np.zeros(n, dtype=np.int64)

    mean32 = np.ascontiguousarray(mean.T, dtype=np.float32)
    cluster = variance_split(mean32.T.astype(np.float64), clusters)
    packet = cluster * contexts + context
    packet_layer = ((packet << 2) | layer).astype(np.uint16)
    return SceneArrays(
        mean=mean32,
        log_scale=np.ascontiguousarray(log_scale.T, dtype=np.float32),
        quat=np.ascontiguousarray(q.T, dtype=np.float32),
        opacity_logit=np.ascontiguousarray(logit, dtype=np.float32),
        color=np.ascontiguousarray(col.T, dtype=np.float32),
        temporal=np.ascontiguousarray(temporal.T, dtype=np.float32),
        packet_layer=packet_layer,
        num_clusters=clusters,
        num_contexts=contexts,
        rank=rank,
        sh_degree=sh_degree,
    )


def make_refinement(scene: SceneArrays, index: int = 0, stream: int = 4, scale: float = 1.0) -> np.ndarray:
    """Three refinement levels of a scene: float32 [3][11 + C][N].

    Level j draws N(0, sigma 2^-(j-1)) per row with sigma = 0.01 (position
    residual), 0.1 (log-scale), 0.1 (quaternion), 0.5 (opacity logit) and
    0.05 (colour), times ``scale``.  The two residual position levels of
    Eq. (1) (delta^(2), delta^(3)) ride on levels 1 and 2; level 3 carries no
    position residual."""
    rng = _rng(index, stream)
    n = scene.n
    C = 3 if scene.sh_degree == 0 else 12
    sig = np.concatenate([np.full(3, 0.01), np.full(3, 0.1), np.full(4, 0.1), [0.5], np.full(C, 0.05)])
    out = np.zeros((3, 11 + C, n), np.float64)
    for j in range(3):
        out[j] = rng.normal(0.0, 1.0, size=(11 + C, n)) * (sig * scale * 2.0 ** -j)[:, None]
    out[2, :3] = 0.0
    return np.ascontiguousarray(out, dtype=np.float32)


def ring_camera(width: int, height: int, theta: float = 0.0, radius: float = 3.0,
                fov_x_deg: float = 60.0, near: float = 0.01) -> CameraArrays:
    """Pinhole camera on a ring of the given radius around the origin, looking
    at the origin with world up +y; OpenCV frame (x right, y down, z forward).
    Rows of R_cw are (right, down, forward); t_cw = -R_cw C."""
    centre = np.array([radius * math.sin(theta), 0.0, -radius * math.cos(theta)])
    fwd = -centre / np.linalg.norm(centre)
    up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ centre
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return CameraArrays(R_cw=R.astype(np.float32), t_cw=t.astype(np.float32),
                        fx=float(np.float32(f)), fy=float(np.float32(f)),
                        cx=float(np.float32(width / 2.0)), cy=float(np.float32(height / 2.0)),
                        width=int(width), height=int(height), near=float(np.float32(near)))


def make_camera(width: int, height: int, **kw) -> CameraArrays:
    return ring_camera(width, height, **kw)


def make_codes(kind: str, lo: float, hi: float, num_states: int, num_packets: int,
               layers: int, index: int = 0, stream: int = 1) -> np.ndarray:
    """Delivery-state codes [W][P] uint8.

    * ``bernoulli``: each packet present with probability ``lo`` (layer 0 only).
    * ``bernoulli_uniform``: per state p_w ~ U[lo, hi], packets ~ Bernoulli(p_w).
    * ``present_depth``: per state p_w ~ U[lo, hi], packets ~ Bernoulli(p_w),
      prefix depth ~ UniformInt{0..layers-1}.
    * ``binomial_ramp``: present fraction f_w rising linearly from lo to hi over
      the states; per packet the number of kept layers ~ Binomial(layers, f_w).
    """
    rng = _rng(index, stream)
    W, P = num_states, num_packets
    if kind == "bernoulli":
        codes = (rng.random((W, P)) < lo).astype(np.uint8)
    elif kind == "bernoulli_uniform":
        p = rng.uniform(lo, hi, size=W)
        codes = (rng.random((W, P)) < p[:, None]).astype(np.uint8)
    elif kind == "present_depth":
        p = rng.uniform(lo, hi, size=W)
        present = rng.random((W, P)) < p[:, None]
        depth = rng.integers(0, layers, size=(W, P))
        codes = np.where(present, depth + 1, 0).astype(np.uint8)
    elif kind == "binomial_ramp":
        f = lo + (hi - lo) * np.arange(W) / max(W - 1, 1)
        codes = rng.binomial(layers, f[:, None], size=(W, P)).astype(np.uint8)
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(codes)


def temporal_basis(t: float, rank: int) -> np.ndarray:
    """Synthetic shared temporal basis b_{t,r} = t^r, r = 1..R (the learned
    basis of Eq. (1) is replaced by monomials; t = 0 gives a static scene)."""
    return np.array([t ** (r + 1) for r in range(rank)], dtype=np.float32)


def perturb_scene(scene: SceneArrays, sigma: float = 0.01, index: int = 0,
                  stream: int = 2) -> SceneArrays:
    """Add N(0, sigma) to every learned parameter array (draw order: mean,
    log_scale, quat, opacity_logit, color, temporal)."""
    rng = _rng(index, stream)

    def noisy(a):
        return (a.astype(np.float64) + rng.normal(0.0, sigma, size=a.shape)).astype(np.float32)

    return replace(scene, mean=noisy(scene.mean), log_scale=noisy(scene.log_scale),
                   quat=noisy(scene.quat), opacity_logit=noisy(scene.opacity_logit),
                   color=noisy(scene.color), temporal=noisy(scene.temporal))


def near_identity_affines(num_clusters: int, sigma: float = 0.05, index: int = 0,
                          stream: int = 5) -> np.ndarray:
    """Per-cluster affines A_c = [I + E | t] ([C][12], row-major 3x4) with E
    ~ N(0, sigma) and t ~ N(0, 2 sigma): random cluster motions near the
    identity, for the A_{c,t} term of Eq. (1)."""
    rng = _rng(index, stream)
    E = rng.normal(0.0, sigma, size=(num_clusters, 3, 3))
    t = rng.normal(0.0, 2.0 * sigma, size=(num_clusters, 3, 1))
    A = np.concatenate([np.eye(3)[None] + E, t], axis=2)
    return np.ascontiguousarray(A.reshape(num_clusters, 12), dtype=np.float32)


def permute_gaussians(scene: SceneArrays, perm: np.ndarray) -> SceneArrays:
    """Reorder the storage of the Gaussians (perm[k] = old index of new k)."""
    take = lambda a: np.ascontiguousarray(a[..., perm])  # noqa: E731
    return replace(scene, mean=take(scene.mean), log_scale=take(scene.log_scale),
                   quat=take(scene.quat), opacity_logit=take(scene.opacity_logit),
                   color=take(scene.color), temporal=take(scene.temporal),
                   packet_layer=take(scene.packet_layer))


def subscene(n: int = 256, width: int = 64, height: int = 64, states: int = 8,
             log_scale_mean: float = -3.0, index: int = 4, stream: int = 3,
             background=(0.25, 0.5, 0.75)) -> Workload:
    """Small scene with the 250k-Gaussian training workload's distributions
    (SH-1 colour, 4 layers, 32x32 packets) for finite-difference checks."""
    scene = make_scene(n, 32, 32, 4, "sh1", index=index, stream=stream)
    if log_scale_mean != -3.0:
        scene = replace(scene, log_scale=(scene.log_scale + np.float32(log_scale_mean + 3.0)))
    cam = ring_camera(width, height)
    codes = make_codes("present_depth", 0.3, 1.0, states, scene.num_packets, 4,
                       index=index, stream=stream + 10)
    return Workload(name=f"sub{n}_{width}x{height}", index=index, scene=scene, camera=cam,
                    codes=codes, basis=temporal_basis(0.5, scene.rank), t=0.5,
                    background=np.asarray(background, dtype=np.float32))


def make_workload(name: str, background=(0.0, 0.0, 0.0), t: float = 0.5,
                  n: Optional[int] = None, states: Optional[int] = None) -> Workload:
    """Build a named workload.  ``n``/``states`` override the sizes (smaller
    instances of the same recipe for tests)."""
    r = WORKLOADS[name]
    idx = r["index"]
    nn = r["n"] if n is None else n
    scene = make_scene(nn, r["clusters"], r["contexts"], r["layers"], r["color"], index=idx)
    cam = ring_camera(r["width"], r["height"])
    W = r["states"] if states is None else states
    kind, lo, hi = r["masks"]
    codes = make_codes(kind, lo, hi, W, scene.num_packets, r["layers"], index=idx)
    return Workload(name=name, index=idx, scene=scene, camera=cam, codes=codes,
                    basis=temporal_basis(t, scene.rank), t=t,
                    background=np.asarray(background, dtype=np.float32),
                    batch=r.get("batch", 0), total_states=r.get("total_states", 0))


# Counterfactual-utility sweeps (Eq. (3)-(4)): completion groups and the
# contexts each group is evaluated in.  ``scene`` names the workload whose
# scene and camera are used.
UTILITY_WORKLOADS = {
    # one group per cluster of the 1M-Gaussian 64x16 scene, 16 contexts each
    "g1m_540p_utility_64groups_16contexts": dict(scene="g1m_540p_32768states_psnr", groups_per_cluster=1,
                                                 contexts_per_group=16, p_lo=0.2, p_hi=1.0, stream=6),
    # the 250k 4-layer scene: one (packet, layer) group per cluster, 8 contexts each
    "g250k_800px_utility_32groups_8contexts": dict(scene="g250k_800px_64states", groups_per_cluster=1,
                                                   contexts_per_group=8, p_lo=0.3, p_hi=1.0, stream=6),
}


@dataclass
class UtilityWorkload:
    base: Workload
    group_pl: np.ndarray       # uint16 [G]: (packet << 2) | layer
    codes: np.ndarray          # uint8 [J][P]: the contexts m
    context_group: np.ndarray  # int32 [J]


def make_utility_contexts(num_clusters: int, num_contexts: int, layers: int, groups_per_cluster: int,
                          contexts_per_group: int, p_lo: float, p_hi: float, index: int, stream: int):
    """Groups: per cluster, ``groups_per_cluster`` distinct random packets of
    that cluster, each with a random layer.  Contexts: per group, states drawn
    as in ``make_codes`` (p_w ~ U[p_lo, p_hi], packets ~ Bernoulli(p_w), prefix
    depth ~ UniformInt{0..layers-1}), then the group's packet set to prefix
    depth exactly the group's layer (its prerequisites delivered, the group
    itself not)."""
    rng = _rng(index, stream)
    P = num_clusters * num_contexts
    gp, gl = [], []
    for c in range(num_clusters):
        ks = rng.choice(num_contexts, size=groups_per_cluster, replace=False)
        for k in ks:
            gp.append(c * num_contexts + int(k))
            gl.append(int(rng.integers(0, layers)))
    G = len(gp)
    J = G * contexts_per_group
    pw = rng.uniform(p_lo, p_hi, size=J)
    present = rng.random((J, P)) < pw[:, None]
    depth = rng.integers(0, layers, size=(J, P))
    codes = np.where(present, depth + 1, 0).astype(np.uint8)
    group = np.repeat(np.arange(G, dtype=np.int32), contexts_per_group)
    codes[np.arange(J), np.asarray(gp)[group]] = np.asarray(gl, dtype=np.uint8)[group]
    group_pl = ((np.asarray(gp, dtype=np.uint32) << 2) | np.asarray(gl, dtype=np.uint32)).astype(np.uint16)
    return group_pl, np.ascontiguousarray(codes), group


def make_utility_workload(name: str, background=(0.0, 0.0, 0.0)) -> UtilityWorkload:
    r = UTILITY_WORKLOADS[name]
    base = make_workload(r["scene"], background=background)
    rb = WORKLOADS[r["scene"]]
    gpl, codes, cg = make_utility_contexts(rb["clusters"], rb["contexts"], rb["layers"], r["groups_per_cluster"],
                                           r["contexts_per_group"], r["p_lo"], r["p_hi"], rb["index"], r["stream"])
    return UtilityWorkload(base=base, group_pl=gpl, codes=codes, context_group=cg)

