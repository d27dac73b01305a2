"""Hand-built scenes for closed-form pins (plain arrays, no renderer arithmetic)."""

import math

import numpy as np

from synth import CameraArrays, SceneArrays, ring_camera


def scene_from_lists(means, log_scales, quats=None, logits=None, colors=None, temporal=None,
                     packet_layer=None, clusters=1, contexts=1, rank=2, sh_degree=0,
                     cluster_affine=None):
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = means.shape[0]
    ls = np.broadcast_to(np.asarray(log_scales, np.float64), (n, 3)) if np.ndim(log_scales) < 2 \
        else np.asarray(log_scales, np.float64)
    q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)) if quats is None else np.asarray(quats, np.float64).reshape(n, 4)
    lg = np.zeros(n) if logits is None else np.asarray(logits, np.float64).reshape(n)
    nc = 3 if sh_degree == 0 else 12
    col = np.full((n, nc), 0.5) if colors is None else np.asarray(colors, np.float64).reshape(n, nc)
    tc = np.zeros((n, 3 * rank)) if temporal is None else np.asarray(temporal, np.float64).reshape(n, 3 * rank)
    pl = np.zeros(n, np.uint16) if packet_layer is None else np.asarray(packet_layer, np.uint16)
    return SceneArrays(mean=np.ascontiguousarray(means.T, np.float32),
                       log_scale=np.ascontiguousarray(np.asarray(ls).T, np.float32),
                       quat=np.ascontiguousarray(q.T, np.float32),
                       opacity_logit=np.ascontiguousarray(lg, np.float32),
                       color=np.ascontiguousarray(col.T, np.float32),
                       temporal=np.ascontiguousarray(tc.T, np.float32),
                       packet_layer=pl, num_clusters=clusters, num_contexts=contexts, rank=rank,
                       sh_degree=sh_degree,
                       cluster_affine=None if cluster_affine is None else np.asarray(cluster_affine, np.float32))


def logit(o):
    return math.log(o / (1.0 - o))


def centred_camera(width=32, height=32, cx=None, cy=None):
    """Ring camera at theta = 0 (centre (0,0,-3), looking along +z) whose
    principal point may be moved, e.g. onto a pixel centre."""
    cam = ring_camera(width, height)
    return CameraArrays(R_cw=cam.R_cw, t_cw=cam.t_cw, fx=cam.fx, fy=cam.fy,
                        cx=cam.cx if cx is None else float(np.float32(cx)),
                        cy=cam.cy if cy is None else float(np.float32(cy)),
                        width=width, height=height, near=cam.near)


def overlap_scene(n=12, seed=7, sh_degree=1, rank=2, spread=0.15, log_scale=-2.2):
    """A few Gaussians crowded near the optical axis so that they overlap and
    occlude each other (used for gradient checks)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-spread, spread, size=(n, 3))
    ls = rng.normal(log_scale, 0.25, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    lg = rng.normal(0.5, 1.0, size=n)
    nc = 3 if sh_degree == 0 else 12
    col = rng.uniform(0, 1, size=(n, 3)) if sh_degree == 0 else rng.normal(0, 0.3, size=(n, nc))
    tc = rng.normal(0, 0.05, size=(n, 3 * rank))
    pl = ((rng.integers(0, 4, size=n) << 2) | rng.integers(0, 4, size=n)).astype(np.uint16)
    return scene_from_lists(means, ls, q, lg, col, tc, pl, clusters=2, contexts=2, rank=rank,
                            sh_degree=sh_degree)
