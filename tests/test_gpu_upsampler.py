"""GPU learned upsampler against the FP64 upsampler oracle, through the C ABI.

Forward and gradients are BF16 on MFMA with FP32 accumulation: compared to
the FP64 oracle by relative L2 error (network residual 2e-2, gradients 3e-2
per layer), with exact identities where no BF16 arithmetic is involved (the
untrained network is bilinear upsampling)."""
import numpy as np
import pytest

import scenegen
from oracle import upsampler as U

pytestmark = pytest.mark.gpu


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _bf16_round(x):
    import torch
    return torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


def _random_params(seed):
    rng = np.random.default_rng(seed)
    params = U.init_params(seed)
    params[3] = (rng.normal(scale=0.03, size=params[3][0].shape), rng.normal(scale=0.01, size=64))
    params = [(w, rng.normal(scale=0.02, size=b.shape)) for (w, b) in params]
    flat = np.concatenate([np.concatenate([w.reshape(-1), b]) for (w, b) in params])
    return params, flat.astype(np.float32)


def _inputs(n, h, w, seed):
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0, 1, size=(n, h, w, 3)).astype(np.float32)
    depth = rng.uniform(1, 20, size=(n, h, w)).astype(np.float32)
    return rgb, depth


def test_param_roundtrip_and_count(gpu_renderer):
    assert gpu_renderer.up_num_params() == sum(w.size + b.size for w, b in U.init_params(0))
    _, flat = _random_params(1)
    gpu_renderer.up_set(flat)
    np.testing.assert_array_equal(gpu_renderer.up_get(), flat)


def test_untrained_network_is_bilinear(gpu_renderer):
    import torch
    gpu_renderer.up_init(3)
    rgb, depth = _inputs(2, 12, 20, 4)
    out_rgb, out_d = gpu_renderer.up_forward(torch.as_tensor(rgb).cuda(), torch.as_tensor(depth).cuda())
    x0 = U.make_input(rgb.astype(np.float64), depth.astype(np.float64))
    ref = U.bilinear_up(x0)
    np.testing.assert_allclose(out_rgb.cpu().numpy(), ref[..., :3], atol=2e-6)
    np.testing.assert_allclose(out_d.cpu().numpy(), ref[..., 3] * U.DEPTH_SCALE, rtol=2e-6)


@pytest.mark.parametrize("n,h,w", [(2, 12, 20), (1, 17, 45), (3, 8, 32)])
def test_forward_matches_oracle(gpu_renderer, n, h, w):
    import torch
    params, flat = _random_params(10 + h)
    gpu_renderer.up_set(flat)
    rgb, depth = _inputs(n, h, w, 5 + h)
    out_rgb, out_d = gpu_renderer.up_forward(torch.as_tensor(rgb).cuda(), torch.as_tensor(depth).cuda())
    x0 = U.make_input(rgb.astype(np.float64), depth.astype(np.float64))
    pred, _ = U.forward(x0, params)
    got = np.concatenate([out_rgb.cpu().numpy(), out_d.cpu().numpy()[..., None] / U.DEPTH_SCALE],
                         axis=-1)
    skip = U.bilinear_up(x0)
    err = _rel_l2(got - skip, pred - skip)
    print(f"forward n={n} {h}x{w}: residual rel L2 {err:.2e}, max abs {np.abs(got - pred).max():.2e}")
    assert err < 2e-2


def test_gradients_match_oracle(gpu_renderer):
    import torch
    params, flat = _random_params(21)
    gpu_renderer.up_set(flat)
    n, h, w = 2, 12, 20
    rgb, depth = _inputs(n, h, w, 22)
    rng = np.random.default_rng(23)
    t_rgb = rng.uniform(0, 1, size=(n, 4 * h, 4 * w, 3)).astype(np.float32)
    t_d = rng.uniform(1, 20, size=(n, 4 * h, 4 * w)).astype(np.float32)
    loss, g = gpu_renderer.up_grads(*[torch.as_tensor(a).cuda() for a in (rgb, depth, t_rgb, t_d)])
    x0 = U.make_input(rgb.astype(np.float64), depth.astype(np.float64))
    target = U.make_input(t_rgb.astype(np.float64), t_d.astype(np.float64))
    pred, acts = U.forward(x0, params)
    ref_loss = U.loss(pred, target)
    grads = U.backward(pred, target, acts, params)
    assert loss == pytest.approx(ref_loss, rel=1e-2)
    off = 0
    for li, (dw, db) in enumerate(grads):
        gw = g[off:off + dw.size].reshape(dw.shape)
        off += dw.size
        gb = g[off:off + db.size]
        off += db.size
        ew, eb = _rel_l2(gw, dw), _rel_l2(gb, db)
        print(f"layer {li + 1}: dW rel L2 {ew:.2e}, db rel L2 {eb:.2e}")
        assert ew < 3e-2 and eb < 3e-2


def test_training_lowers_loss_and_fallback_paths(gpu_renderer):
    import torch
    sc = scenegen.make_scene(1)
    sid = gpu_renderer.upload_scene(sc)
    train = scenegen.sampled_cameras(1, 256, seed=1)
    gpu_renderer.up_init(0)
    curve = gpu_renderer.up_train([sid] * 256, train["poses"], train["intrinsics"], 640, 480,
                                  batch=16, steps=48, lr=2e-3)
    print("loss curve", curve[:4], curve[-4:])
    assert np.isfinite(curve).all()
    assert curve[-8:].mean() < curve[:8].mean()
    ev = scenegen.make_cameras(1)
    P, K = ev["poses"][:8], ev["intrinsics"][:8]
    ids = [sid] * 8
    full = gpu_renderer.render(ids, P, K, 640, 480, alpha=False)
    # every camera falls back: the output is the full-resolution render, bitwise
    rgb, depth, score, nf = gpu_renderer.render_upsampled(ids, P, K, 640, 480, threshold=-1.0)
    assert nf == 8
    assert bool((rgb == full[0]).all()) and bool((depth == full[1]).all())
    # no camera falls back: the upsampled output, scored
    rgb, depth, score, nf = gpu_renderer.render_upsampled(ids, P, K, 640, 480)
    assert nf == 0 and bool(torch.isfinite(rgb).all()) and bool((score >= 0).all())
    ps = gpu_renderer.frame_psnr(rgb, full[0]).cpu().numpy()
    ref = U.psnr(rgb.cpu().numpy().astype(np.float64), full[0].cpu().numpy().astype(np.float64))
    np.testing.assert_allclose(ps, ref, atol=1e-3)
    print("psnr", ps)
    # some cameras fall back: exactly those are the full-resolution render,
    # written into their own frames; the others keep the upsampled images
    sc_np = score.cpu().numpy()
    thr = float(np.sort(sc_np)[3])
    rgb2, depth2, score2, nf2 = gpu_renderer.render_upsampled(ids, P, K, 640, 480, threshold=thr)
    flagged = ~(score2.cpu().numpy() <= thr)
    assert nf2 == int(flagged.sum()) and 0 < nf2 < 8
    for c in range(8):
        ref_rgb, ref_d = (full[0][c], full[1][c]) if flagged[c] else (rgb[c], depth[c])
        assert bool((rgb2[c] == ref_rgb).all()) and bool((depth2[c] == ref_d).all()), c
    gpu_renderer.release_scene(sid)


def test_checkpoint_restores_training_state_exactly(gpu_renderer, tmp_path):
    """Save after a few Adam steps, load into a second context: the same
    further steps give bitwise the same weights in both (parameters, both
    Adam moments and the step count are restored)."""
    import paper_2510_15352_amd as gs
    sc = scenegen.tiny_scene(2000, 5, sh_degree=1, spread=1.0)
    train = scenegen.sampled_cameras(1, 32, seed=3)
    sid = gpu_renderer.upload_scene(sc)
    pose = train["poses"].copy()
    pose[:, :, :3] = np.eye(3, dtype=np.float32)
    pose[:, :, 3] = np.random.default_rng(0).uniform(-0.3, 0.3, size=(32, 3))
    pose[:, 2, 3] -= 4.0
    intr = np.tile(np.array([[80.0, 80.0, 32.0, 24.0]], np.float32), (32, 1))
    gpu_renderer.up_init(3)
    gpu_renderer.up_train([sid] * 32, pose, intr, 64, 48, batch=8, steps=4, lr=3e-3)
    path = str(tmp_path / "up.ckpt")
    gpu_renderer.up_save(path)
    gpu_renderer.up_train([sid] * 32, pose, intr, 64, 48, batch=8, steps=3, lr=3e-3)
    a = gpu_renderer.up_get()
    other = gs.Renderer(0)
    try:
        sid2 = other.upload_scene(sc)
        other.up_load(path)
        other.up_train([sid2] * 32, pose, intr, 64, 48, batch=8, steps=3, lr=3e-3)
        b = other.up_get()
        with pytest.raises(gs.GsError):
            other.up_load(str(tmp_path / "missing.ckpt"))
    finally:
        other.close()
    gpu_renderer.release_scene(sid)
    assert np.array_equal(a, b)
