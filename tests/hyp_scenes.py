"""Hypothesis strategies for tiny scenes with the cases random workloads rarely
hit: Gaussians off screen or behind the near plane, degenerate (sub-pixel or
very elongated) scales, exact depth ties, clusters with non-identity affines,
and arbitrary delivery codes.  Plain arrays only (no renderer arithmetic)."""

import numpy as np
from hypothesis import strategies as st

from synth import near_identity_affines
from tests.scenes_for_tests import centred_camera, scene_from_lists


@st.composite
def tiny_scenes(draw, max_n=24):
    n = draw(st.integers(1, max_n))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    spread = draw(st.sampled_from([0.3, 0.8, 2.5]))  # 2.5: many Gaussians off screen
    means = rng.uniform(-spread, spread, size=(n, 3))
    if draw(st.booleans()):  # exact depth ties: equal z for groups of Gaussians
        means[:, 2] = np.round(means[:, 2] * 2.0) / 2.0
    if draw(st.booleans()):  # some behind the camera (z < -3) or on its plane
        k = rng.integers(0, n)
        means[k, 2] = draw(st.sampled_from([-3.0, -3.5, -2.995]))
    ls_mean = draw(st.sampled_from([-6.0, -3.0, -1.8]))  # -6: footprints below a pixel
    log_scales = rng.normal(ls_mean, 0.3, size=(n, 3))
    if draw(st.booleans()):  # very elongated
        log_scales[:, 0] += 2.0
    q = rng.normal(size=(n, 4))
    logits = rng.normal(0.5, 1.5, size=n)
    sh = draw(st.sampled_from([0, 1]))
    cols = rng.uniform(0, 1, size=(n, 3)) if sh == 0 else rng.normal(0, 0.3, size=(n, 12))
    temporal = rng.normal(0, 0.05, size=(n, 6))
    clusters, contexts = 2, 2
    pl = ((rng.integers(0, clusters * contexts, size=n) << 2) | rng.integers(0, 4, size=n)).astype(np.uint16)
    aff = near_identity_affines(clusters, index=seed % 1000) if draw(st.booleans()) else None
    scene = scene_from_lists(means, log_scales, q, logits, cols, temporal, pl, clusters=clusters,
                             contexts=contexts, sh_degree=sh, cluster_affine=aff)
    width = draw(st.sampled_from([16, 40, 72]))
    height = draw(st.sampled_from([16, 24, 56]))
    cam = centred_camera(width, height)
    W = draw(st.integers(1, 6))
    codes = rng.integers(0, 6, size=(W, clusters * contexts)).astype(np.uint8)  # 5 acts as 4
    t = draw(st.sampled_from([0.0, 0.5, 1.0]))
    basis = np.array([t, t * t], np.float32)
    return scene, cam, basis, codes
