"""Batched partial-delivery Gaussian splatting on AMD MI355X (gfx950).

Renders one dynamic Gaussian scene (clustered Gaussians with affine +
low-rank temporal motion, one base and three refinement layers per cluster)
under many incomplete delivery states in one batched launch, forward and
backward, through the hand-written HIP kernels of ``libdgs.so``.
"""

from .render import (CapturedRender, StreamPipeline, Camera, GaussianScene, Renderer, RenderFunction, distortion,  # noqa: F401
                     render, risk_adjusted, sample_states, channels_to_device, CHANNEL_DTYPE, Objective,
                     ObjectiveFunction, OBJECTIVE_WEIGHTS, L1Loss, L1Function, l1_loss, render_noalloc)
from .autotune import Autotuner  # noqa: F401
from ._abi import DgsError, lib  # noqa: F401
