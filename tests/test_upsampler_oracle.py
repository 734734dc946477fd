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
