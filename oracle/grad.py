"""FP64 dense formulation of the masked render in plain PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY.  Its autograd is the reference gradient: the exact
derivative of the render with every discrete decision frozen at the branch
the FP64 forward takes (culling, sort order, the 1/255 skip, the 0.99 cap,
the stop after T < 1e-4, the SH clamp at 0, the Jacobian clamp, the L1 sign).
Depth only orders, so it carries no gradient.

The formulation is independent of ``oracle.c``'s per-pixel loop: for each
pixel the alphas of all Gaussians, in the global (FP32 depth bits, index)
order, form one dense row; skipped, absent and post-stop entries are zeroed;
transmittance is an exclusive cumulative product.  The two FP64 forwards
agree to rounding, which pins each against coding slips in the other.

Sections followed: Sec. 3, Eq. (1) (deformation); Sec. 6 (many delivery
states rendered from one scene, FP32 rasterisation -- here FP64).
"""

from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import mirror_f32

SH_C0 = 0.28209479177387814
SH_C1 = 0.4886025119029199
ALPHA_MIN = 1.0 / 255.0
T_STOP = 1e-4

PARAMS = ("mean", "log_scale", "quat", "opacity_logit", "color", "temporal")


def _quat_rot(q):
    qn = q / torch.sqrt((q * q).sum(0, keepdim=True))
    w, x, y, z = qn[0], qn[1], qn[2], qn[3]
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)  # [N,3,3]
    return R


def project(p: dict, scene, cam, basis):
    """Per-Gaussian FP64 quantities as differentiable tensors: u, v, conic
    (A, B, C), opacity o, colour [N,3]."""
    mean, log_scale, quat = p["mean"], p["log_scale"], p["quat"]
    n = mean.shape[1]
    mu = mean
    if scene.cluster_affine is not None:
        aff = torch.as_tensor(np.asarray(scene.cluster_affine, np.float64)).reshape(-1, 3, 4)
        cl = torch.as_tensor((scene.packet_layer.astype(np.int64) >> 2) // scene.num_contexts)
        Ai = aff[cl]  # [N,3,4]
        mu = torch.einsum("nkj,jn->kn", Ai[:, :, :3], mean) + Ai[:, :, 3].T
    for r in range(scene.rank):
        mu = mu + float(basis[r]) * p["temporal"][3 * r:3 * r + 3]
    if "offset" in p:  # delivered position residual levels, after the deformation
        mu = mu + p["offset"]
    Rc = torch.as_tensor(np.asarray(cam.R_cw, np.float64))
    tc = torch.as_tensor(np.asarray(cam.t_cw, np.float64))
    P = Rc @ mu + tc[:, None]
    X, Y, Z = P[0], P[1], P[2]
    fx, fy = float(cam.fx), float(cam.fy)
    Rq = _quat_rot(quat)
    S = torch.exp(2.0 * log_scale).T  # [N,3]
    Sig = Rq @ torch.diag_embed(S) @ Rq.transpose(1, 2)
    Sc = Rc[None] @ Sig @ Rc.T[None]
    limx = 1.3 * cam.width / (2.0 * fx)
    limy = 1.3 * cam.height / (2.0 * fy)
    tx = torch.clamp(X / Z, -limx, limx)
    ty = torch.clamp(Y / Z, -limy, limy)
    zero = torch.zeros_like(Z)
    J = torch.stack([torch.stack([fx / Z, zero, -fx * tx / Z], -1),
                     torch.stack([zero, fy / Z, -fy * ty / Z], -1)], -2)  # [N,2,3]
    S2 = J @ Sc @ J.transpose(1, 2)
    a = S2[:, 0, 0] + 0.3
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + 0.3
    det = a * c - b * b
    u = fx * X / Z + float(cam.cx)
    v = fy * Y / Z + float(cam.cy)
    o = torch.sigmoid(p["opacity_logit"])
    if scene.sh_degree == 0:
        col = p["color"].T
    else:
        C = -(Rc.T @ tc)
        d = mu - C[:, None]
        d = d / torch.sqrt((d * d).sum(0, keepdim=True))
        k = p["color"].reshape(4, 3, n)
        val = 0.5 + SH_C0 * k[0] + SH_C1 * (-d[1] * k[1] + d[2] * k[2] - d[0] * k[3])
        col = torch.clamp(val, min=0.0).T
    return dict(u=u, v=v, A=c / det, B=-b / det, C=a / det, o=o, col=col)


def params_from_scene(scene, requires_grad=True) -> dict:
    return {k: torch.tensor(np.asarray(getattr(scene, k), np.float64), requires_grad=requires_grad)
            for k in PARAMS}


def render_dense(scene, cam, basis, codes, background, pixels=None, params=None,
                 chunk: int = 256):
    """FP64 render as a differentiable function of ``params``.

    Returns (image [W][K][3] float64 tensor, params).  ``pixels``: int [K][2]
    (x, y) or None for all pixels row-major."""
    if params is None:
        params = params_from_scene(scene)
    mir = mirror_f32(scene, cam, basis)
    n = scene.mean.shape[1]
    valid = mir["valid"]
    order = np.lexsort((np.arange(n), mir["zbits"].astype(np.int64)))
    order = order[valid[order]]
    g = project(params, scene, cam, basis)
    if pixels is None:
        ys, xs = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
        pixels = np.stack([xs.reshape(-1), ys.reshape(-1)], 1)
    pixels = np.asarray(pixels, np.int64).reshape(-1, 2)
    idx = torch.as_tensor(order)
    u, v = g["u"][idx], g["v"][idx]
    A, B, C, o, col = g["A"][idx], g["B"][idx], g["C"][idx], g["o"][idx], g["col"][idx]
    pl = scene.packet_layer.astype(np.int64)[order]
    codes = np.asarray(codes, np.int64)
    pres = torch.as_tensor((pl[None, :] & 3) < codes[:, pl >> 2])  # [W, n_sorted]
    bg = torch.as_tensor(np.asarray(background, np.float64))
    outs = []
    for s0 in range(0, pixels.shape[0], chunk):
        pix = torch.as_tensor(pixels[s0:s0 + chunk] + 0.5, dtype=torch.float64)
        dx = u[None, :] - pix[:, 0:1]
        dy = v[None, :] - pix[:, 1:2]
        q = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy
        al = torch.clamp(o * torch.exp(-0.5 * q), max=0.99)  # [K, n]
        keep = (al.detach() >= ALPHA_MIN)
        per_state = []
        for w in range(codes.shape[0]):
            m = keep & pres[w][None, :]
            ae = torch.where(m, al, torch.zeros_like(al))
            with torch.no_grad():
                Tafter = torch.cumprod(1.0 - ae, dim=1)
                stop = Tafter < T_STOP
                # entries after the first stop are frozen out
                after = torch.cumsum(stop.to(torch.int64), dim=1) - stop.to(torch.int64) > 0
            ae = torch.where(after, torch.zeros_like(ae), ae)
            onem = 1.0 - ae
            Tincl = torch.cumprod(onem, dim=1)
            Tbefore = torch.cat([torch.ones_like(Tincl[:, :1]), Tincl[:, :-1]], dim=1)
            wgt = Tbefore * ae
            Cc = wgt @ col + Tincl[:, -1:] * bg[None, :] if ae.shape[1] else bg[None, :].expand(ae.shape[0], 3)
            per_state.append(Cc)
        outs.append(torch.stack(per_state, 0))
    return torch.cat(outs, 1), params


def gradients(scene, cam, basis, codes, background, grad_image, pixels=None) -> dict:
    """Reference parameter gradients for an upstream image gradient
    ``grad_image`` ([W][K][3] matching ``pixels``, or [W][H][Wd][3]).
    Only Gaussians that reach alpha >= 1/255 (less a small margin) at one of
    the pixels take part; every other Gaussian's gradient is exactly zero
    because it is skipped at every pixel."""
    n = scene.mean.shape[1]
    if pixels is None:
        ys, xs = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
        pixels = np.stack([xs.reshape(-1), ys.reshape(-1)], 1)
    pixels = np.asarray(pixels, np.int64).reshape(-1, 2)
    gi = torch.as_tensor(np.asarray(grad_image, np.float64).reshape(codes.shape[0], -1, 3))
    # candidates: Gaussians that reach the skip threshold somewhere in the pixel set
    with torch.no_grad():
        g0 = project(params_from_scene(scene, False), scene, cam, basis)
        cand = np.zeros(n, dtype=bool)
        pix = torch.as_tensor(pixels + 0.5, dtype=torch.float64)
        for s0 in range(0, pixels.shape[0], 64):
            pp = pix[s0:s0 + 64]
            dx = g0["u"][None, :] - pp[:, 0:1]
            dy = g0["v"][None, :] - pp[:, 1:2]
            q = g0["A"] * dx * dx + 2.0 * g0["B"] * dx * dy + g0["C"] * dy * dy
            al = g0["o"] * torch.exp(-0.5 * q)
            cand |= (al >= ALPHA_MIN * 0.5).any(0).numpy()
    sel = np.nonzero(cand)[0]
    sub = dataclasses.replace(scene, mean=scene.mean[:, sel], log_scale=scene.log_scale[:, sel],
                              quat=scene.quat[:, sel], opacity_logit=scene.opacity_logit[sel],
                              color=scene.color[:, sel], temporal=scene.temporal[:, sel],
                              packet_layer=scene.packet_layer[sel])
    img, params = render_dense(sub, cam, basis, codes, background, pixels)
    (img * gi).sum().backward()
    out = {}
    for k in PARAMS:
        full = np.zeros(np.asarray(getattr(scene, k)).shape, dtype=np.float64)
        full[..., sel] = params[k].grad.numpy()
        out[k] = full
    return out


def render_dense_refined(scene, refine, cam, basis, codes, background, pixels=None, base=None, levels=None):
    """FP64 render of a scene with refinement levels (Sec. 3) as a
    differentiable function of the base parameters ``base`` (dict of PARAMS)
    and the levels ``levels`` ([3][rows][N]).  Each state w renders its
    decoded scene: Gaussian i, delivered to depth d, carries base + level 1 +
    ... + level d, and the position residual level 1 + ... + level d after the
    deformation.  Discrete decisions come from the FP32 decoded scene
    (``oracle.refined_scene``) and are frozen.  Returns [W][K][3]."""
    from . import refined_scene
    codes = np.asarray(codes, np.uint8)
    if base is None:
        base = params_from_scene(scene, requires_grad=False)
    if levels is None:
        levels = torch.tensor(np.asarray(refine, np.float64))
    pl = scene.packet_layer.astype(np.int64)
    out = []
    for w in range(codes.shape[0]):
        depth = np.minimum(codes[w][pl >> 2].astype(np.int64), 4) - 1
        add = sum(levels[j] * torch.as_tensor((depth >= j + 1).astype(np.float64)) for j in range(3))
        p = {"mean": base["mean"], "temporal": base["temporal"], "log_scale": base["log_scale"] + add[3:6],
             "quat": base["quat"] + add[6:10], "opacity_logit": base["opacity_logit"] + add[10],
             "color": base["color"] + add[11:], "offset": add[0:3]}
        dec = refined_scene(scene, refine, codes[w])
        img, _ = render_dense(dec, cam, basis, codes[w:w + 1], background, pixels, params=p)
        out.append(img[0])
    return torch.stack(out, 0)


def gradients_refined(scene, refine, cam, basis, codes, background, grad_image, pixels=None) -> dict:
    """Reference gradients of a scene with refinement levels for an upstream
    image gradient: autograd of ``render_dense_refined``.  Returns the base
    parameter gradients (PARAMS) and ``refine`` [3][rows][N]."""
    codes = np.asarray(codes, np.uint8)
    W = codes.shape[0]
    base = params_from_scene(scene)
    lv = torch.tensor(np.asarray(refine, np.float64), requires_grad=True)
    out = {k: np.zeros(np.asarray(getattr(scene, k)).shape, dtype=np.float64) for k in PARAMS}
    out["refine"] = np.zeros(lv.shape, dtype=np.float64)
    if W == 0:
        return out
    gi = torch.as_tensor(np.asarray(grad_image, np.float64).reshape(W, -1, 3))
    img = render_dense_refined(scene, refine, cam, basis, codes, background, pixels, base, lv)
    (img * gi).sum().backward()
    for k in PARAMS:
        if base[k].grad is not None:
            out[k] = base[k].grad.numpy().copy()
    if lv.grad is not None:
        out["refine"] = lv.grad.numpy().copy()
    return out


def l1_loss(image, target) -> float:
    """Mean |C - target| over every element (the plain L1 training loss), in
    FP64; ``target`` broadcasts against ``image``."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    return float(np.abs(d).mean())


def l1_loss_grad(image, target) -> np.ndarray:
    """d/dC of mean |C - target| over every element (sign(0) = 0)."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    return np.sign(d) / d.size
