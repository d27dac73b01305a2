"""Counterfactual render utility (paper Sec. 5, Eq. (3)-(4)) -- TEST
INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

* ``ssim``: structural similarity of two images with the usual 11x11 Gaussian
  window (sigma 1.5), constants (0.01)^2 and (0.03)^2, zero padding outside
  the image ('same' output), averaged over pixels and channels.  Written as
  the definition: every window statistic is an explicit weighted sum over the
  121 offsets, in FP64.
* ``distortion``: D = MSE + lambda (1 - SSIM), the distortion the paper fixes
  for its objective (Sec. 4, lambda = 0.20); used here for Eq. (3).
* ``paired_states``: m and m u g for a completion group g = (packet, layer):
  m holds the packet at prefix depth exactly `layer`, m u g at `layer + 1`.
* ``deltas``: Delta_g(m) = D(I, R(m)) - D(I, R(m u g)) (Eq. (3)) from full
  renders of both states by the FP64 oracle renderer.
* ``risk_adjusted``: ((1 - a) E[Delta] + a Q_q(Delta)) / (1 + b Std(Delta))
  (Eq. (4)), with the quantile by linear interpolation between order
  statistics and the population standard deviation.
"""

from __future__ import annotations

import numpy as np

SSIM_RADIUS = 5
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window() -> np.ndarray:
    """11x11 Gaussian weights (sigma 1.5), normalised to sum 1."""
    r = np.arange(-SSIM_RADIUS, SSIM_RADIUS + 1, dtype=np.float64)
    g = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def _window_mean(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum_{dy,dx} w[dy,dx] x[y+dy, x+dx] with x = 0 outside the image;
    ``x`` is [H, W, C]."""
    H, Wd = x.shape[:2]
    R = SSIM_RADIUS
    pad = np.zeros((H + 2 * R, Wd + 2 * R) + x.shape[2:], dtype=np.float64)
    pad[R:R + H, R:R + Wd] = x
    out = np.zeros_like(x, dtype=np.float64)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            out += w[dy + R, dx + R] * pad[R + dy:R + dy + H, R + dx:R + dx + Wd]
    return out


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Per-pixel, per-channel SSIM of images [H, W, C] (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = ssim_window()
    mx, my = _window_mean(x, w), _window_mean(y, w)
    sxx = _window_mean(x * x, w) - mx * mx
    syy = _window_mean(y * y, w) - my * my
    sxy = _window_mean(x * y, w) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def ssim(x: np.ndarray, y: np.ndarray) -> float:
    return float(ssim_map(x, y).mean())


def mse(x: np.ndarray, y: np.ndarray) -> float:
    d = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return float((d * d).mean())


def distortion(x: np.ndarray, y: np.ndarray, lam: float = 0.20) -> float:
    """D = MSE + lam (1 - SSIM) between an image and the reference."""
    return mse(x, y) + lam * (1.0 - ssim(x, y))


def paired_states(contexts: np.ndarray, packet: int, layer: int):
    """(m, m u g) code rows for the completion group (packet, layer); every
    context must hold the packet at prefix depth exactly ``layer``."""
    m = np.asarray(contexts, dtype=np.uint8)
    if not np.all(m[:, packet] == layer):
        raise ValueError("a context does not hold the group's packet at its prefix depth")
    mg = m.copy()
    mg[:, packet] = layer + 1
    return m, mg


def deltas(scene, cam, basis, contexts, packet: int, layer: int, reference, background, lam: float = 0.20,
           refine=None):
    """Delta_g(m) of Eq. (3) for every context row (FP64 oracle renders).
    With ``refine`` (attribute refinement levels, Sec. 3) each state renders
    its decoded scene (``oracle.render_refined``): adding g moves the packet's
    Gaussians from depth ``layer - 1`` to depth ``layer``."""
    from . import render, render_refined

    m, mg = paired_states(contexts, packet, layer)
    if refine is None:
        a = render(scene, cam, basis, m, background)["image"]
        b = render(scene, cam, basis, mg, background)["image"]
    else:
        a = render_refined(scene, refine, cam, basis, m, background)["image"]
        b = render_refined(scene, refine, cam, basis, mg, background)["image"]
    return np.array([distortion(a[j], reference, lam) - distortion(b[j], reference, lam) for j in range(len(m))])


def quantile_linear(values, q: float) -> float:
    """Order statistics x_(0) <= ... <= x_(n-1); position h = (n - 1) q;
    value x_(floor h) + (h - floor h) (x_(floor h + 1) - x_(floor h))."""
    v = sorted(float(x) for x in values)
    h = (len(v) - 1) * q
    lo = int(np.floor(h))
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (h - lo) * (v[hi] - v[lo])


def risk_adjusted(values, alpha: float = 0.25, beta: float = 0.05, q: float = 0.10) -> dict:
    """Eq. (4) over the contexts of one group, with its three statistics."""
    v = np.asarray(values, dtype=np.float64)
    mean = float(v.mean())
    std = float(np.sqrt(((v - mean) ** 2).mean()))
    qv = quantile_linear(v, q)
    return {"mean": mean, "quantile": qv, "std": std,
            "risk_adjusted": ((1.0 - alpha) * mean + alpha * qv) / (1.0 + beta * std)}
