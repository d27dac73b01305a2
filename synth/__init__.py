"""Seeded synthetic inputs shared by the renderer's tests, its bench and the oracle.

This package draws random numbers and does bookkeeping only (cluster ids,
packet ids, camera pose, delivery-state codes).  None of the renderer's
arithmetic lives here: the oracle and the GPU path both consume these arrays
and share nothing else.
"""

from .workloads import (  # noqa: F401
    SceneArrays,
    CameraArrays,
    Workload,
    WORKLOADS,
    make_scene,
    make_refinement,
    make_camera,
    ring_camera,
    make_codes,
    temporal_basis,
    variance_split,
    perturb_scene,
    subscene,
    make_workload,
    permute_gaussians,
    near_identity_affines,
    UTILITY_WORKLOADS,
    UtilityWorkload,
    make_utility_contexts,
    make_utility_workload,
)
