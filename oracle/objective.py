"""Packet-conditioned rendering objective (paper Sec. 4, Eq. (2)) -- TEST
INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

    L = E_w[D_w] + lambda_c CVaR_alpha(D) + lambda_r R + lambda_t F
        + lambda_m M + lambda_a D_anchor

with the constants the paper locks (D = MSE + 0.20 (1 - SSIM), lambda_c =
0.30, alpha = 0.05, lambda_r = 0, lambda_t = 0.10, lambda_m = 2.0, anchor
weight 0.50).  The batch is a list of rendered images, each compared with a
target image; index lists give each image its role:

* ``expect``: partial delivery states; E_w[D_w] is their mean D and
  CVaR_alpha the mean of the worst alpha fraction of their D values (upper
  tail; the Rockafellar-Uryasev value of the empirical distribution: the
  largest floor(alpha n) values count fully, the next one with the fractional
  remainder, all divided by alpha n).
* ``anchor``: complete-prefix states, supervised directly (mean D).
* ``mono``: pairs (a, b) where state b grows a's prefix; M is the mean of
  max(0, D_b - D_a), a quality regression as the prefix grows.
* ``temporal``: pairs (a, b) of one world rendered at two times; F is the
  mean over pairs of the mean squared error between the rendered change
  I_b - I_a and the target change G_b - G_a.
* R (rate proxy) has weight 0 in the locked configuration and does not
  depend on the rendered images; it is left out.

Everything is FP64 in plain PyTorch CPU ops; the SSIM window sums are one
``conv2d`` with the 11x11 Gaussian (sigma 1.5, zero padding, 'same' size), so
the image gradient of L is autograd's.
"""

from __future__ import annotations

import numpy as np
import torch

from . import utility as U

LOCKED = dict(lambda_ssim=0.20, lambda_c=0.30, alpha=0.05, lambda_t=0.10, lambda_m=2.0, lambda_a=0.50)


def _window() -> torch.Tensor:
    return torch.from_numpy(U.ssim_window()).to(torch.float64)


def ssim_t(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Mean SSIM over pixels and channels of images [H, W, C] (FP64 tensors)."""
    C = x.shape[-1]
    w = _window()[None, None].expand(C, 1, -1, -1).contiguous()
    X = x.permute(2, 0, 1)[None]
    Y = y.permute(2, 0, 1)[None]
    R = U.SSIM_RADIUS

    def wm(t):
        return torch.nn.functional.conv2d(t, w, padding=R, groups=C)

    mx, my = wm(X), wm(Y)
    sxx = wm(X * X) - mx * mx
    syy = wm(Y * Y) - my * my
    sxy = wm(X * Y) - mx * my
    s = ((2 * mx * my + U.SSIM_C1) * (2 * sxy + U.SSIM_C2)) / \
        ((mx * mx + my * my + U.SSIM_C1) * (sxx + syy + U.SSIM_C2))
    return s.mean()


def distortion_t(x: torch.Tensor, y: torch.Tensor, lambda_ssim: float = 0.20) -> torch.Tensor:
    """D = MSE + lambda (1 - SSIM) of one image against its target."""
    return ((x - y) ** 2).mean() + lambda_ssim * (1.0 - ssim_t(x, y))


def cvar_upper(d: torch.Tensor, alpha: float) -> torch.Tensor:
    """Mean of the worst alpha fraction of the values d (upper tail): with
    a = alpha n, k = floor(a), the k largest count 1 each and the (k+1)-th
    the remainder a - k; the sum is divided by a.  Ties are broken by lower
    position first (any choice gives the same value)."""
    n = d.numel()
    if n == 0:
        return d.sum() * 0.0
    a = alpha * n
    k = int(np.floor(a))
    # descending by value, ascending position among equal values
    dv = d.detach()
    order = sorted(range(n), key=lambda i: (-float(dv[i]), i))
    wts = torch.zeros(n, dtype=torch.float64)
    for r in range(min(k, n)):
        wts[order[r]] = 1.0
    if k < n and a - k > 0:
        wts[order[k]] = a - k
    return (wts * d).sum() / a


def objective(images, targets, target_of, expect, anchor=(), mono=(), temporal=(), weights=None,
              grad: bool = True) -> dict:
    """Eq. (2) of a batch.  images [K][H][W][3], targets [T][H][W][3] (any
    float dtype), target_of [K], index lists / pairs as in the module header.
    Returns loss and its parts (E, CVaR, F, M, anchor), D per image and,
    with ``grad``, dL/d images [K][H][W][3] (float64 numpy)."""
    wts = dict(LOCKED)
    wts.update(weights or {})
    x = torch.tensor(np.asarray(images, np.float64), requires_grad=grad)
    g = torch.tensor(np.asarray(targets, np.float64))
    tgt = [int(t) for t in target_of]
    K = x.shape[0]
    D = torch.stack([distortion_t(x[k], g[tgt[k]], wts["lambda_ssim"]) for k in range(K)]) if K else \
        torch.zeros(0, dtype=torch.float64)
    zero = x.sum() * 0.0
    e_idx = [int(i) for i in expect]
    De = D[e_idx] if e_idx else torch.zeros(0, dtype=torch.float64)
    E = De.mean() if e_idx else zero
    cv = cvar_upper(De, wts["alpha"]) if e_idx else zero
    a_idx = [int(i) for i in anchor]
    A = D[a_idx].mean() if a_idx else zero
    M = torch.stack([torch.relu(D[int(b)] - D[int(a)]) for a, b in mono]).mean() if len(mono) else zero
    if len(temporal):
        F = torch.stack([(((x[int(b)] - x[int(a)]) - (g[tgt[int(b)]] - g[tgt[int(a)]])) ** 2).mean()
                         for a, b in temporal]).mean()
    else:
        F = zero
    L = E + wts["lambda_c"] * cv + wts["lambda_t"] * F + wts["lambda_m"] * M + wts["lambda_a"] * A
    L_, E_, cv_, F_, M_, A_ = (float(v.detach()) for v in (L, E, cv, F, M, A))
    out = dict(loss=L_, E=E_, cvar=cv_, F=F_, M=M_, anchor=A_,
               D=D.detach().numpy().copy())
    if grad:
        L.backward()
        out["grad"] = x.grad.numpy().copy()
    return out
