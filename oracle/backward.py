"""FP64 gradients of the splat renderer's outputs -- TEST INFRASTRUCTURE ONLY.

Only `tests/` may import this module. It shares no code with the GPU path.

The paper builds its scenes by optimising 3D Gaussian splats whose renders
are differentiable (Sec. 2.3: splats rasterised differentiably, fitted to
images; Sec. 3.1: 3DGS optimised from the reconstructed points). The
gradient computed here is the derivative of the plain FP64 definition of the
forward render (the one `gs_oracle.c` computes, restated below with the same
FP32-valued constants) with respect to every scene parameter, for given
upstream gradients of the outputs:

    L = sum_cameras sum_pixels  gR . RGB + gD * depth + gA * alpha

Forward, per camera (pose camera-to-world [R_cw | C], intrinsics fx fy cx cy):
  p = R_wc mu + t_wc; Gaussians with z <= near are dropped;
  Sigma = R(q/|q|) diag(s)^2 R^T; J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]]
  with tx, ty = x/z, y/z clamped to 1.3x the image half-extent;
  Sigma' = J W Sigma W^T J^T + 0.3 I; conic Q = Sigma'^-1;
  (u, v) = (fx x/z + cx, fy y/z + cy);
  colour = max(0, sum_lm k_lm Y_lm(d) + 0.5), d = (mu - C)/|mu - C|, real SH
  with the Condon-Shortley phase from the associated Legendre recurrence;
  per pixel centre: alpha_g = min(0.99, o_g exp(-1/2 delta^T Q delta)),
  skipped (alpha taken as 0) below 1/255; Gaussians in (z, index) order;
  T_g = prod_{j<g} (1 - alpha_j); Gaussian g is included while
  T_g (1 - alpha_g) >= 1e-4 (the walk stops at the first that is not);
  w_g = alpha_g T_g for included ones;
  RGB = sum w c + T_final bg, depth = sum w z / sum w (0 if sum w = 0),
  alpha = sum w.

The walk is evaluated densely (every pixel against every Gaussian in front,
which is the same candidate set as the footprint-bounded walk since a
Gaussian outside its footprint has alpha < 1/255) with cumulative products
along the depth order, and differentiated by reverse-mode automatic
differentiation in float64 (torch, CPU). The discrete decisions (near
plane, skip, stop, the alpha clamp, the tangent clamp, the colour clamp)
are taken as in the forward pass and held fixed: the derivative is that of
the branch the forward pass takes (zero through a clamp that is active).
The SH basis goes through the azimuth atan2(y, x), whose derivative is
undefined on the world z axis: directions exactly along it are not used.
"""
from __future__ import annotations

import math

import numpy as np
import torch

F32 = lambda x: float(np.float32(x))  # noqa: E731
ALPHA_MAX = F32(0.99)
ALPHA_MIN = F32(1.0 / 255.0)
T_MIN = F32(1e-4)
LOWPASS = F32(0.3)
TAN_CLAMP = F32(1.3)

_DT = torch.float64


def _assoc_legendre(l, m, x):
    """P_l^m(x), m >= 0, with the Condon-Shortley phase (three-term recurrence)."""
    pmm = torch.ones_like(x)
    if m > 0:
        s = torch.sqrt(torch.clamp((1.0 - x) * (1.0 + x), min=0.0))
        fact = 1.0
        for _ in range(m):
            pmm = pmm * (-fact) * s
            fact += 2.0
    if l == m:
        return pmm
    pmmp1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pmmp1
    pll = pmmp1
    for ll in range(m + 2, l + 1):
        pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m)
        pmm, pmmp1 = pmmp1, pll
    return pll


def sh_basis(deg, d):
    """Real SH Y_lm(d / |d|) for l <= deg, l-major with m = -l..l: [N, (deg+1)^2]."""
    dn = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    x, y, z = dn.unbind(-1)
    phi = torch.atan2(y, x)
    cols = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) /
                          math.factorial(l + am))
            P = _assoc_legendre(l, am, z)
            if m == 0:
                cols.append(K * P)
            elif m > 0:
                cols.append(math.sqrt(2.0) * K * P * torch.cos(am * phi))
            else:
                cols.append(math.sqrt(2.0) * K * P * torch.sin(am * phi))
    return torch.stack(cols, dim=-1)


def _quat_rot(q):
    qn = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = qn.unbind(-1)
    return torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1).reshape(-1, 3, 3)


def project(params, deg, pose, intr, W, H, near):
    """Per-Gaussian projection in float64: dict of u, v, conic (A, B, C),
    opacity, rgb [N, 3], z and the in-front mask."""
    means, scales, quats, opacity, sh = params
    pose = torch.as_tensor(np.asarray(pose, np.float32).reshape(3, 4), dtype=_DT)
    fx, fy, cx, cy = (float(np.float32(v)) for v in np.asarray(intr).reshape(4))
    Rwc = pose[:, :3].T
    C = pose[:, 3]
    t = -(Rwc @ C)
    p = means @ Rwc.T + t
    x, y, z = p.unbind(-1)
    front = (z > near).detach()
    # keep the projection finite for Gaussians behind the near plane (dropped)
    zs = torch.where(front, z, torch.ones_like(z))
    Rq = _quat_rot(quats)
    Sig = (Rq * (scales * scales)[:, None, :]) @ Rq.transpose(1, 2)
    lxn, lxp = -TAN_CLAMP * cx / fx, TAN_CLAMP * (W - cx) / fx
    lyn, lyp = -TAN_CLAMP * cy / fy, TAN_CLAMP * (H - cy) / fy
    tx = torch.clamp(x / zs, lxn, lxp)
    ty = torch.clamp(y / zs, lyn, lyp)
    zero = torch.zeros_like(zs)
    J = torch.stack([fx / zs, zero, -fx * tx / zs, zero, fy / zs, -fy * ty / zs], -1).reshape(-1, 2, 3)
    T = J @ Rwc
    Sp = T @ Sig @ T.transpose(1, 2)
    a = Sp[:, 0, 0] + LOWPASS
    b = 0.5 * (Sp[:, 0, 1] + Sp[:, 1, 0])
    c = Sp[:, 1, 1] + LOWPASS
    det = a * c - b * b
    u = fx * x / zs + cx
    v = fy * y / zs + cy
    Y = sh_basis(deg, means - C)
    rgb = torch.clamp(torch.einsum("nk,nkc->nc", Y, sh) + 0.5, min=0.0)
    return dict(u=u, v=v, A=c / det, B=-b / det, C=a / det, o=opacity, rgb=rgb, z=z, front=front)


def composite(pr, W, H, bg, rows=None):
    """Dense front-to-back walk of every pixel centre of the given rows over
    the Gaussians in front, in (z, index) order. Returns rgb [R, W, 3],
    depth [R, W], alpha [R, W] and the per-pair decision masks (for tests)."""
    idx = torch.nonzero(pr["front"]).reshape(-1)
    zf = pr["z"].detach()[idx].numpy()
    order = idx[np.lexsort((idx.numpy(), zf))]
    u, v = pr["u"][order], pr["v"][order]
    A, B, C = pr["A"][order], pr["B"][order], pr["C"][order]
    o, rgb, z = pr["o"][order], pr["rgb"][order], pr["z"][order]
    rows = list(range(H)) if rows is None else list(rows)
    jj, ii = np.meshgrid(np.asarray(rows, np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    px = torch.as_tensor(ii.reshape(-1) + 0.5, dtype=_DT)[:, None]
    py = torch.as_tensor(jj.reshape(-1) + 0.5, dtype=_DT)[:, None]
    dx, dy = px - u[None, :], py - v[None, :]
    power = -0.5 * (A * dx * dx + 2.0 * B * dx * dy + C * dy * dy)
    al = torch.clamp(o * torch.exp(power), max=ALPHA_MAX)
    keep = (al >= ALPHA_MIN).detach()
    al = torch.where(keep, al, torch.zeros_like(al))
    one_m = 1.0 - al
    t_incl = torch.cumprod(one_m, dim=1)
    incl = (t_incl >= T_MIN).detach()
    t_excl = torch.cat([torch.ones_like(t_incl[:, :1]), t_incl[:, :-1]], dim=1)
    w = al * t_excl * incl
    acc_rgb = w @ rgb
    acc_z = w @ z
    acc_w = w.sum(dim=1)
    t_fin = torch.prod(torch.where(incl, one_m, torch.ones_like(one_m)), dim=1)
    bgv = torch.as_tensor(np.asarray(bg, np.float64), dtype=_DT)
    out_rgb = acc_rgb + t_fin[:, None] * bgv[None, :]
    has = acc_w > 0
    depth = torch.where(has, acc_z / torch.where(has, acc_w, torch.ones_like(acc_w)),
                        torch.zeros_like(acc_w))
    R = len(rows)
    return (out_rgb.reshape(R, W, 3), depth.reshape(R, W), acc_w.reshape(R, W),
            dict(keep=keep, incl=incl, order=order))


def _params(scene, grad):
    keys = ("means", "scales", "quats", "opacity", "sh")
    out = []
    for k in keys:
        t = torch.as_tensor(np.asarray(scene[k], np.float32).astype(np.float64), dtype=_DT)
        if k == "sh":
            t = t.reshape(len(scene["opacity"]), -1, 3)
        out.append(t.requires_grad_(grad))
    return out


def render(scene, pose, intr, W, H, near=0.2, bg=(0.0, 0.0, 0.0)):
    """The forward definition above, in float64 (numpy outputs)."""
    with torch.no_grad():
        pr = project(_params(scene, False), int(scene["sh_degree"]), pose, intr, W, H,
                     F32(near))
        n_front = max(int(pr["front"].sum()), 1)
        rows_per = max(1, (1 << 21) // (n_front * W))
        parts = [composite(pr, W, H, bg, range(r0, min(H, r0 + rows_per)))[:3]
                 for r0 in range(0, H, rows_per)]
    return tuple(torch.cat([p[i] for p in parts]).numpy() for i in range(3))


def grads(scene, poses, intrs, W, H, g_rgb, g_depth=None, g_alpha=None, near=0.2,
          bg=(0.0, 0.0, 0.0), max_pairs=1 << 21):
    """Gradients of L (module docstring) with respect to means [N, 3], scales
    [N, 3], quats [N, 4], opacity [N] and sh [N, K, 3], summed over the
    cameras; g_rgb [n, H, W, 3], g_depth / g_alpha [n, H, W] or None.
    Returns a dict of float64 arrays."""
    params = _params(scene, True)
    deg = int(scene["sh_degree"])
    n = len(poses)
    for c in range(n):
        pr = project(params, deg, poses[c], intrs[c], W, H, F32(near))
        names = ("u", "v", "A", "B", "C", "o", "rgb", "z")
        leaf = {k: pr[k].detach().clone().requires_grad_(True) for k in names}
        leaf["front"] = pr["front"]
        n_front = max(int(pr["front"].sum()), 1)
        rows_per = max(1, max_pairs // (n_front * W))
        for r0 in range(0, H, rows_per):
            rows = range(r0, min(H, r0 + rows_per))
            rgb, depth, alpha, _ = composite(leaf, W, H, bg, rows)
            sl = slice(r0, r0 + len(rows))
            loss = (rgb * torch.as_tensor(np.asarray(g_rgb[c][sl], np.float64))).sum()
            if g_depth is not None:
                loss = loss + (depth * torch.as_tensor(np.asarray(g_depth[c][sl], np.float64))).sum()
            if g_alpha is not None:
                loss = loss + (alpha * torch.as_tensor(np.asarray(g_alpha[c][sl], np.float64))).sum()
            loss.backward()
        outs, gouts = [], []
        for k in names:
            if leaf[k].grad is not None:
                outs.append(pr[k])
                gouts.append(leaf[k].grad)
        torch.autograd.backward(outs, gouts)
    keys = ("means", "scales", "quats", "opacity", "sh")
    return {k: (p.grad.numpy().copy() if p.grad is not None else np.zeros(p.shape))
            for k, p in zip(keys, params)}


def loss_value(scene, poses, intrs, W, H, g_rgb, g_depth=None, g_alpha=None, near=0.2,
               bg=(0.0, 0.0, 0.0), params=None):
    """L for the given scene (or float64 parameter arrays), no gradient:
    for finite-difference pins. Also returns the decision masks per camera."""
    deg = int(scene["sh_degree"])
    with torch.no_grad():
        ps = _params(scene, False) if params is None else [
            torch.as_tensor(np.asarray(a, np.float64)) for a in params]
        if params is not None:
            ps[4] = ps[4].reshape(len(ps[3]), -1, 3)
        total, masks = 0.0, []
        for c in range(len(poses)):
            pr = project(ps, deg, poses[c], intrs[c], W, H, F32(near))
            rgb, depth, alpha, m = composite(pr, W, H, bg)
            total += float((rgb * torch.as_tensor(np.asarray(g_rgb[c], np.float64))).sum())
            if g_depth is not None:
                total += float((depth * torch.as_tensor(np.asarray(g_depth[c], np.float64))).sum())
            if g_alpha is not None:
                total += float((alpha * torch.as_tensor(np.asarray(g_alpha[c], np.float64))).sum())
            masks.append((pr["front"].numpy().copy(), m["keep"].numpy().copy(),
                          m["incl"].numpy().copy(), m["order"].numpy().copy(),
                          (torch.abs(pr["rgb"]) > 0).numpy().copy()))
    return total, masks
