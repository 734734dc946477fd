"""FP64 reference of the learned 4x upsampler -- TEST INFRASTRUCTURE ONLY.

The network (a workload definition, not from the paper): the low-resolution
render (RGB + depth / 10) is the 4-channel input x0 at h x w; four 3x3
convolutions with zero padding, 4 -> 32 -> 32 -> 32 -> 64 channels, ReLU
after the first three; the 64 output channels are rearranged by a 4x pixel
shuffle into 4 channels at 4h x 4w and added to the bilinear 4x upsampling of
x0. Loss: mean over pixels of sum_c w_c (pred_c - target_c)^2 with w = (1, 1,
1, 0.1).

Layouts are NHWC; weights are [Cout][3][3][Cin]. Pixel shuffle (factor r):
out[n, r*y + i, r*x + j, c] = in[n, y, x, c*r*r + i*r + j]. Bilinear 4x with
half-pixel centres: source coordinate (t + 0.5) / 4 - 0.5, clamped at 0,
neighbours clamped to the last row/column.

Training step: Adam with bias correction (Kingma & Ba, 2015) on every
parameter, a cosine learning-rate schedule from lr0 at the first step to
lr_min at the last, and, for the upsampled render's fallback, a per-frame
confidence score (mean squared forward difference of the four input
channels along x and y).

Everything is written from these definitions with numpy loops over the nine
taps; the tests pin it against torch.nn.functional and torch.optim.Adam
(float64, CPU), central finite differences, closed forms and explicit loops.
"""
from __future__ import annotations

import numpy as np

R = 4
CH = (4, 32, 32, 32, 64)
LOSS_W = np.array([1.0, 1.0, 1.0, 0.1])
DEPTH_SCALE = 10.0
TAPS = [(ky, kx) for ky in range(3) for kx in range(3)]


def pad1(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))


def conv3x3(x, w, b):
    """y[n, i, j, o] = b[o] + sum_{ky,kx,c} xpad[n, i+ky, j+kx, c] w[o, ky, kx, c]."""
    n, h, wd, ci = x.shape
    xp = pad1(x)
    y = np.broadcast_to(b, (n, h, wd, w.shape[0])).astype(np.float64).copy()
    for ky, kx in TAPS:
        y += xp[:, ky:ky + h, kx:kx + wd, :] @ w[:, ky, kx, :].T
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 w.r.t. x, w and b given dL/dy."""
    n, h, wd, ci = x.shape
    xp = pad1(x)
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky, kx in TAPS:
        dxp[:, ky:ky + h, kx:kx + wd, :] += dy @ w[:, ky, kx, :]
        dw[:, ky, kx, :] = np.einsum("nijo,nijc->oc", dy, xp[:, ky:ky + h, kx:kx + wd, :])
    return dxp[:, 1:-1, 1:-1, :], dw, dy.sum(axis=(0, 1, 2))


def pixel_shuffle(y, r=R):
    n, h, w, c = y.shape
    co = c // (r * r)
    t = y.reshape(n, h, w, co, r, r)            # [n, y, x, c, i, j]
    return t.transpose(0, 1, 4, 2, 5, 3).reshape(n, h * r, w * r, co)


def pixel_unshuffle(z, r=R):
    n, H, W, co = z.shape
    t = z.reshape(n, H // r, r, W // r, r, co)  # [n, y, i, x, j, c]
    return t.transpose(0, 1, 3, 5, 2, 4).reshape(n, H // r, W // r, co * r * r)


def _bilinear_axis(n_in, r=R):
    t = (np.arange(n_in * r) + 0.5) / r - 0.5
    t = np.maximum(t, 0.0)
    i0 = np.floor(t).astype(np.int64)
    i0 = np.minimum(i0, n_in - 1)
    i1 = np.minimum(i0 + 1, n_in - 1)
    return i0, i1, t - i0


def bilinear_up(x, r=R):
    n, h, w, c = x.shape
    y0, y1, fy = _bilinear_axis(h, r)
    x0, x1, fx = _bilinear_axis(w, r)
    top = x[:, y0, :, :] * (1 - fy)[None, :, None, None] + x[:, y1, :, :] * fy[None, :, None, None]
    return top[:, :, x0, :] * (1 - fx)[None, None, :, None] + top[:, :, x1, :] * fx[None, None, :, None]


def init_params(seed=0):
    """He-uniform weights, zero biases; the last layer starts at zero so the
    untrained network is exactly the bilinear upsampler."""
    rng = np.random.default_rng(seed)
    params = []
    for li in range(4):
        ci, co = CH[li], CH[li + 1]
        bound = np.sqrt(6.0 / (9 * ci))
        w = rng.uniform(-bound, bound, size=(co, 3, 3, ci))
        if li == 3:
            w[:] = 0.0
        params.append((w, np.zeros(co)))
    return params


def forward(x0, params):
    acts = [x0]
    a = x0
    for li, (w, b) in enumerate(params):
        z = conv3x3(a, w, b)
        a = np.maximum(z, 0.0) if li < 3 else z
        acts.append(a)
    pred = bilinear_up(x0) + pixel_shuffle(acts[-1])
    return pred, acts


def loss(pred, target):
    d = pred - target
    return float((d * d * LOSS_W).sum(axis=-1).mean())


def backward(pred, target, acts, params):
    """Gradients of loss() w.r.t. every (w, b); returns [(dw, db)] per layer."""
    npix = pred.shape[0] * pred.shape[1] * pred.shape[2]
    dpred = 2.0 * (pred - target) * LOSS_W / npix
    dy = pixel_unshuffle(dpred)
    grads = [None] * 4
    for li in range(3, -1, -1):
        w, _ = params[li]
        dx, dw, db = conv3x3_backward(acts[li], w, dy)
        grads[li] = (dw, db)
        if li > 0:
            dy = dx * (acts[li] > 0)
    return grads


def make_input(rgb, depth):
    """[n, h, w, 4] network input from an RGB + depth render."""
    return np.concatenate([rgb, depth[..., None] / DEPTH_SCALE], axis=-1)


def psnr(pred_rgb, target_rgb):
    """Per-frame PSNR in dB of RGB clamped to [0, 1]."""
    a = np.clip(pred_rgb, 0.0, 1.0)
    b = np.clip(target_rgb, 0.0, 1.0)
    mse = ((a - b) ** 2).reshape(a.shape[0], -1).mean(axis=1)
    return 10.0 * np.log10(1.0 / np.maximum(mse, 1e-12))


# ------------------------------------------------------------ training step --

ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(p, g, m, v, step, lr, b1=ADAM_B1, b2=ADAM_B2, eps=ADAM_EPS):
    """One Adam update (Kingma & Ba, 2015): step is the 1-based index of this
    update. m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2; with the
    bias-corrected moments m_hat = m / (1 - b1^step), v_hat = v / (1 -
    b2^step), p <- p - lr m_hat / (sqrt(v_hat) + eps). Returns new (p, m, v)
    (float64 arrays)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** step)
    v_hat = v / (1.0 - b2 ** step)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def cosine_lr(s, steps, lr0, lr_min):
    """Learning rate of optimisation step s (0-based) of `steps`: half a
    cosine period from lr0 at s = 0 down to lr_min at s = steps - 1 (lr0
    throughout when steps == 1)."""
    if steps <= 1:
        return float(lr0)
    return float(lr_min + 0.5 * (lr0 - lr_min) * (1.0 + np.cos(np.pi * s / (steps - 1))))


def confidence_score(x0):
    """Per-frame score of the network input x0 [n, h, w, 4]: the sum over
    channels of the squared forward differences to the right and downward
    neighbours (where they exist), divided by the h w pixels of the frame."""
    x0 = np.asarray(x0, np.float64)
    n, h, w, _ = x0.shape
    dx = x0[:, :, 1:, :] - x0[:, :, :-1, :]
    dy = x0[:, 1:, :, :] - x0[:, :-1, :, :]
    return ((dx * dx).sum(axis=(1, 2, 3)) + (dy * dy).sum(axis=(1, 2, 3))) / (h * w)


def flatten(params):
    """[(w, b)] per layer -> the parameter vector (per layer: w [cout][3][3][cin], then b)."""
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for (w, b) in params])


def unflatten(vec):
    """Inverse of flatten() for the network's layer shapes."""
    out, off = [], 0
    for li in range(4):
        ci, co = CH[li], CH[li + 1]
        nw = co * 9 * ci
        w = np.asarray(vec[off:off + nw], np.float64).reshape(co, 3, 3, ci)
        off += nw
        b = np.asarray(vec[off:off + co], np.float64)
        off += co
        out.append((w, b))
    return out


def train_step(params, m, v, step, x0, target, lr):
    """One optimisation step on a batch: forward, loss, backward, then Adam
    on the parameter vector. params / m / v are parameter vectors; step is
    the 1-based Adam step. Returns (loss, new params, new m, new v)."""
    layers = unflatten(params)
    pred, acts = forward(x0, layers)
    lval = loss(pred, target)
    g = flatten(backward(pred, target, acts, layers))
    p2, m2, v2 = adam_step(params, g, m, v, step, lr)
    return lval, p2, m2, v2
