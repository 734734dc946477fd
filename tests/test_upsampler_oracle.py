"""Pins of the FP64 upsampler oracle: convolution, pixel shuffle and bilinear
upsampling against torch.nn.functional in float64 on the CPU (library
routines), gradients against central finite differences, and the identity
of the untrained network with bilinear upsampling."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import upsampler as U


def nchw(x):
    return torch.from_numpy(np.ascontiguousarray(x.transpose(0, 3, 1, 2)))


def nhwc(t):
    return t.numpy().transpose(0, 2, 3, 1)


def test_conv3x3_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 7, 9, 5))
    w = rng.normal(size=(6, 3, 3, 5))
    b = rng.normal(size=6)
    ref = F.conv2d(nchw(x), torch.from_numpy(w.transpose(0, 3, 1, 2).copy()),
                   torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(U.conv3x3(x, w, b), nhwc(ref), atol=1e-12)


def test_pixel_shuffle_matches_torch_and_inverts():
    rng = np.random.default_rng(1)
    y = rng.normal(size=(2, 3, 5, 64))
    ref = F.pixel_shuffle(nchw(y), 4)
    np.testing.assert_array_equal(U.pixel_shuffle(y), nhwc(ref))
    np.testing.assert_array_equal(U.pixel_unshuffle(U.pixel_shuffle(y)), y)


def test_bilinear_matches_torch():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 6, 7, 4))
    ref = F.interpolate(nchw(x), scale_factor=4, mode="bilinear", align_corners=False)
    np.testing.assert_allclose(U.bilinear_up(x), nhwc(ref), atol=1e-12)


def test_untrained_network_is_bilinear():
    rng = np.random.default_rng(3)
    x0 = rng.uniform(size=(1, 5, 6, 4))
    pred, _ = U.forward(x0, U.init_params(0))
    np.testing.assert_allclose(pred, U.bilinear_up(x0), atol=0)


def test_backward_matches_torch_autograd():
    rng = np.random.default_rng(4)
    params = U.init_params(5)
    params[3] = (rng.normal(scale=0.05, size=params[3][0].shape), rng.normal(size=64) * 0.01)
    params = [(w, rng.normal(scale=0.01, size=b.shape)) for (w, b) in params]
    x0 = rng.uniform(size=(2, 4, 5, 4))
    target = rng.uniform(size=(2, 16, 20, 4))
    pred, acts = U.forward(x0, params)
    grads = U.backward(pred, target, acts, params)
    # the same network in torch (float64), autograd gradients
    tw = [torch.tensor(w.transpose(0, 3, 1, 2).copy(), requires_grad=True) for w, _ in params]
    tb = [torch.tensor(b, requires_grad=True) for _, b in params]
    a = nchw(x0)
    for li in range(4):
        a = F.conv2d(a, tw[li], tb[li], padding=1)
        if li < 3:
            a = torch.relu(a)
    tp = F.interpolate(nchw(x0), scale_factor=4, mode="bilinear", align_corners=False) + \
        F.pixel_shuffle(a, 4)
    d = tp - nchw(target)
    lw = torch.tensor(U.LOSS_W).view(1, 4, 1, 1)
    tl = (d * d * lw).sum(dim=1).mean()
    tl.backward()
    assert float(tl.detach()) == pytest.approx(U.loss(pred, target), rel=1e-12)
    for li in range(4):
        np.testing.assert_allclose(grads[li][0], tw[li].grad.numpy().transpose(0, 2, 3, 1),
                                   rtol=1e-9, atol=1e-14)
        np.testing.assert_allclose(grads[li][1], tb[li].grad.numpy(), rtol=1e-9, atol=1e-14)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(6)
    params = [(w * 0.5, rng.normal(scale=0.05, size=b.shape)) for (w, b) in U.init_params(7)]
    params[3] = (rng.normal(scale=0.05, size=params[3][0].shape), params[3][1])
    x0 = rng.uniform(size=(1, 3, 4, 4))
    target = rng.uniform(size=(1, 12, 16, 4))
    pred, acts = U.forward(x0, params)
    grads = U.backward(pred, target, acts, params)
    h = 1e-6
    for li in range(4):
        w, b = params[li]
        for idx in [tuple(rng.integers(0, s) for s in w.shape) for _ in range(4)]:
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            pp = list(params)
            pp[li] = (wp, b)
            lp = U.loss(U.forward(x0, pp)[0], target)
            pp[li] = (wm, b)
            lm = U.loss(U.forward(x0, pp)[0], target)
            num = (lp - lm) / (2 * h)
            assert grads[li][0][idx] == pytest.approx(num, rel=1e-5, abs=1e-9)


def test_psnr_definition():
    a = np.zeros((1, 4, 4, 3))
    b = np.full((1, 4, 4, 3), 0.1)
    assert U.psnr(a, b)[0] == pytest.approx(20.0)
    assert U.psnr(np.full((1, 2, 2, 3), 2.0), np.ones((1, 2, 2, 3)))[0] == pytest.approx(120.0)


# ------------------------------------------------------------ training step --

def test_adam_matches_torch_optim_adam():
    """Five steps with changing gradients and learning rates against
    torch.optim.Adam (float64, CPU; the library routine of Kingma & Ba)."""
    rng = np.random.default_rng(30)
    p0 = rng.normal(size=257)
    p = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(U.ADAM_B1, U.ADAM_B2), eps=U.ADAM_EPS)
    mine, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step in range(1, 6):
        g = rng.normal(size=p0.shape) * 10.0 ** rng.uniform(-6, 1, size=p0.shape)
        lr = 1e-3 * (1.0 + step)
        for grp in opt.param_groups:
            grp["lr"] = lr
        p.grad = torch.tensor(g)
        opt.step()
        mine, m, v = U.adam_step(mine, g, m, v, step, lr)
        np.testing.assert_allclose(mine, p.detach().numpy(), rtol=1e-13, atol=1e-15)
        st = opt.state[p]
        np.testing.assert_allclose(m, st["exp_avg"].numpy(), rtol=1e-13, atol=0)
        np.testing.assert_allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-13, atol=0)


def test_adam_closed_forms():
    """The first step moves every parameter by lr g / (|g| + eps); a constant
    gradient keeps moving it by exactly that each step (both bias-corrected
    moments equal g and g^2); a zero gradient moves nothing."""
    g = np.array([3.0, -0.5, 1e-3, -2e-5, 0.0])
    p0 = np.array([0.1, 0.2, -0.3, 0.4, 0.5])
    lr = 0.01
    step1 = lr * g / (np.abs(g) + U.ADAM_EPS)
    p, m, v = U.adam_step(p0, g, np.zeros(5), np.zeros(5), 1, lr)
    np.testing.assert_allclose(p, p0 - step1, rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 1e-3 * g * g, rtol=1e-12)
    for k in range(2, 6):
        p, m, v = U.adam_step(p, g, m, v, k, lr)
        np.testing.assert_allclose(p, p0 - k * step1, rtol=0, atol=1e-14)
    assert p[4] == p0[4]


def test_cosine_schedule_closed_forms():
    lr0, lr1, steps = 2e-3, 1e-4, 9
    lrs = [U.cosine_lr(s, steps, lr0, lr1) for s in range(steps)]
    assert lrs[0] == pytest.approx(lr0, rel=1e-15)
    assert lrs[-1] == pytest.approx(lr1, rel=1e-12)
    assert lrs[4] == pytest.approx(0.5 * (lr0 + lr1), rel=1e-12)      # half-way
    assert lrs[2] == pytest.approx(lr1 + (lr0 - lr1) * np.cos(np.pi / 8) ** 2, rel=1e-12)
    assert all(a > b for a, b in zip(lrs, lrs[1:]))
    assert U.cosine_lr(0, 1, lr0, lr1) == lr0


def test_confidence_score_explicit_loop_and_closed_forms():
    rng = np.random.default_rng(31)
    x = rng.normal(size=(2, 3, 5, 4))
    want = []
    for f in range(2):
        s = 0.0
        for y in range(3):
            for xx in range(5):
                for c in range(4):
                    if xx + 1 < 5:
                        s += (x[f, y, xx + 1, c] - x[f, y, xx, c]) ** 2
                    if y + 1 < 3:
                        s += (x[f, y + 1, xx, c] - x[f, y, xx, c]) ** 2
        want.append(s / 15)
    np.testing.assert_allclose(U.confidence_score(x), want, rtol=1e-13)
    # a constant frame scores 0; a ramp a*x in one channel scores h (w-1) a^2 / (h w)
    h, w, a = 6, 7, 0.3
    ramp = np.zeros((1, h, w, 4))
    ramp[0, :, :, 2] = a * np.arange(w)[None, :] + 5.0
    assert U.confidence_score(np.full((1, h, w, 4), 0.7))[0] == 0.0
    assert U.confidence_score(ramp)[0] == pytest.approx(h * (w - 1) * a * a / (h * w), rel=1e-13)


def test_train_step_composition():
    """With a zero learning rate the parameters stay put and the moments are
    those of the finite-difference-pinned gradient; the parameter vector
    layout round-trips."""
    rng = np.random.default_rng(32)
    params = U.init_params(8)
    params[3] = (rng.normal(scale=0.05, size=params[3][0].shape), rng.normal(scale=0.01, size=64))
    vec = U.flatten(params)
    for (w, b), (w2, b2) in zip(params, U.unflatten(vec)):
        np.testing.assert_array_equal(w, w2)
        np.testing.assert_array_equal(b, b2)
    x0 = rng.uniform(size=(1, 3, 4, 4))
    target = rng.uniform(size=(1, 12, 16, 4))
    loss, p, m, v = U.train_step(vec, np.zeros_like(vec), np.zeros_like(vec), 1, x0, target, 0.0)
    pred, acts = U.forward(x0, params)
    g = U.flatten(U.backward(pred, target, acts, params))
    assert loss == U.loss(pred, target)
    np.testing.assert_array_equal(p, vec)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 1e-3 * g * g, rtol=1e-12)
