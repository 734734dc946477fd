"""The no-allocation upsampler forward (gs_upsampler_forward_noalloc, for
callers that cannot allocate device memory) against the allocating entry
point gs_upsampler_forward, through the C ABI: the same kernels on the same
inputs, so the frames must be bitwise equal, on two calls in a row (the
second with a smaller input, after the first left its activations in the
shared scratch array), plus a frame too large for the scratch array, which
must be refused before anything runs."""
import numpy as np
import pytest

from oracle import upsampler as U

pytestmark = pytest.mark.gpu


def _params(seed):
    rng = np.random.default_rng(seed)
    params = U.init_params(seed)
    params[3] = (rng.normal(scale=0.03, size=params[3][0].shape), rng.normal(scale=0.01, size=64))
    params = [(w, rng.normal(scale=0.02, size=b.shape)) for (w, b) in params]
    return params, np.concatenate([np.concatenate([w.reshape(-1), b])
                                   for (w, b) in params]).astype(np.float32)


def _frames(n, h, w, seed):
    import torch
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0, 1, size=(n, h, w, 3)).astype(np.float32)
    depth = rng.uniform(1, 20, size=(n, h, w)).astype(np.float32)
    return rgb, depth, torch.as_tensor(rgb).cuda(), torch.as_tensor(depth).cuda()


def test_noalloc_forward_equals_allocating_forward(gpu_renderer):
    import torch
    params, flat = _params(71)
    gpu_renderer.up_set(flat)
    # 40 frames of 160x120: 16 frames per pass through the 64 MiB scratch
    # (three passes, the last one ragged); then 3 frames of 45x17
    for n, h, w, seed in ((40, 120, 160, 72), (3, 17, 45, 73)):
        print(f"no-alloc forward: n={n} {w}x{h}", flush=True)
        rgb, depth, rgb_d, depth_d = _frames(n, h, w, seed)
        ref_rgb, ref_d = gpu_renderer.up_forward(rgb_d, depth_d)
        out_rgb = torch.full((n, 4 * h, 4 * w, 3), float("nan"), device=rgb_d.device)
        out_d = torch.full((n, 4 * h, 4 * w), float("nan"), device=rgb_d.device)
        gpu_renderer.up_forward_noalloc(rgb_d, depth_d, out_rgb, out_d)
        torch.cuda.synchronize()
        assert torch.equal(out_rgb, ref_rgb) and torch.equal(out_d, ref_d)
        if n <= 3:
            # and both match the FP64 oracle's network to the forward's bar
            x0 = U.make_input(rgb.astype(np.float64), depth.astype(np.float64))
            pred, _ = U.forward(x0, params)
            got = np.concatenate([out_rgb.cpu().numpy(),
                                  out_d.cpu().numpy()[..., None] / U.DEPTH_SCALE], axis=-1)
            skip = U.bilinear_up(x0)
            err = np.linalg.norm((got - skip) - (pred - skip)) / np.linalg.norm(pred - skip)
            print(f"residual rel L2 vs oracle {err:.2e}", flush=True)
            assert err < 2e-2


def test_noalloc_forward_refuses_frames_larger_than_its_scratch(gpu_renderer):
    import torch
    import paper_2510_15352_amd as gs
    _, flat = _params(74)
    gpu_renderer.up_set(flat)
    h, w = 600, 600   # 208 bytes x 360,000 pixels > 64 MiB
    rgb_d = torch.zeros((1, h, w, 3), device="cuda")
    depth_d = torch.ones((1, h, w), device="cuda")
    out_rgb = torch.zeros((1, 4 * h, 4 * w, 3), device="cuda")
    out_d = torch.zeros((1, 4 * h, 4 * w), device="cuda")
    with pytest.raises(gs.GsError) as e:
        gpu_renderer.up_forward_noalloc(rgb_d, depth_d, out_rgb, out_d)
    assert e.value.code == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(out_rgb.abs().max()) == 0.0
