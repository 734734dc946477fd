"""Pins of the FP64 gradient oracle (oracle/backward.py): its forward pass
is the C oracle's render; its gradients match central finite differences of
that forward pass and closed forms for a single Gaussian."""
import math

import numpy as np
import pytest

import oracle
import scenegen
from oracle import backward as B

IDENT_POSE = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)


def _cams(n, seed, W, H, f=18.0):
    rng = np.random.default_rng(seed)
    poses = np.zeros((n, 3, 4), np.float32)
    for c in range(n):
        a = rng.normal(scale=0.15, size=3)
        th = np.linalg.norm(a)
        k = a / th
        Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        poses[c, :, :3] = np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * Kx @ Kx
        poses[c, :, 3] = rng.uniform(-0.2, 0.2, size=3)
    intr = np.tile(np.array([[f, f, W / 2 + 0.3, H / 2 - 0.2]], np.float32), (n, 1))
    return poses, intr


def _upstream(n, W, H, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(n, H, W, 3)), rng.normal(size=(n, H, W)) * 0.1,
            rng.normal(size=(n, H, W)))


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_forward_is_the_c_oracle_render(deg):
    sc = scenegen.tiny_scene(40, 50 + deg, sh_degree=deg, spread=0.8)
    poses, intr = _cams(2, 60 + deg, 24, 18)
    for c in range(2):
        rgb, depth, alpha = B.render(sc, poses[c], intr[c], 24, 18, bg=(0.1, 0.2, 0.3))
        ref = oracle.render(sc, poses[c], intr[c], 24, 18, bg=(0.1, 0.2, 0.3))
        np.testing.assert_allclose(rgb, ref.rgb, atol=1e-12)
        np.testing.assert_allclose(depth, ref.depth, atol=1e-11)
        np.testing.assert_allclose(alpha, ref.alpha, atol=1e-12)


def test_forward_on_workload0_subset():
    sc = scenegen.make_scene(0)
    sub = {k: (v[:1500] if k != "sh_degree" else v) for k, v in sc.items()}
    cams = scenegen.make_cameras(0)
    rgb, depth, alpha = B.render(sub, cams["poses"][0], cams["intrinsics"][0], 64, 48)
    ref = oracle.render(sub, cams["poses"][0], cams["intrinsics"][0], 64, 48)
    np.testing.assert_allclose(rgb, ref.rgb, atol=1e-11)
    np.testing.assert_allclose(alpha, ref.alpha, atol=1e-11)
    np.testing.assert_allclose(depth, ref.depth, rtol=1e-11, atol=1e-11)


def _flat(scene):
    return [np.asarray(scene[k], np.float32).astype(np.float64).copy()
            for k in ("means", "scales", "quats", "opacity", "sh")]


@pytest.mark.parametrize("deg,seed", [(0, 1), (1, 2), (3, 3), (3, 4)])
def test_gradients_match_central_finite_differences(deg, seed):
    W, H = 20, 16
    sc = scenegen.tiny_scene(7, 80 + seed, sh_degree=deg, spread=0.5, log_scale_mean=-1.8)
    sc["opacity"] = np.random.default_rng(seed).uniform(0.3, 0.8, 7).astype(np.float32)
    poses, intr = _cams(2, 90 + seed, W, H)
    gr, gd, ga = _upstream(2, W, H, 100 + seed)
    g = B.grads(sc, poses, intr, W, H, gr, gd, ga, bg=(0.2, 0.1, 0.0))
    rng = np.random.default_rng(200 + seed)
    base = _flat(sc)
    names = ("means", "scales", "quats", "opacity", "sh")
    checked = 0
    for gi, name in enumerate(names):
        arr = base[gi]
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            vals, masks = [], []
            for sgn in (1, -1):
                p = [a.copy() for a in base]
                p[gi][idx] += sgn * h
                v, m = B.loss_value(sc, poses, intr, W, H, gr, gd, ga, bg=(0.2, 0.1, 0.0),
                                    params=p)
                vals.append(v)
                masks.append(m)
            # a discrete decision (skip, stop, order, clamp) between the two
            # evaluations makes the difference quotient meaningless: skip it
            same = all(all(np.array_equal(x, y) for x, y in zip(m0, m1))
                       for m0, m1 in zip(masks[0], masks[1]))
            if not same:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            ad = g[name].reshape(arr.shape)[idx]
            assert ad == pytest.approx(fd, rel=2e-5, abs=2e-6), (name, idx, ad, fd)
            checked += 1
    assert checked >= 24


def test_single_gaussian_closed_forms():
    """One isotropic Gaussian on the optical axis, black background, dL/dRGB
    = 1 on the red channel: RGB_r(p) = c_r alpha(p) where alpha(p) =
    o exp(-q(p)/2) is below the clamp, so dL/do = c_r sum_p alpha(p)/o and
    dL/dk_00,r = Y_00 sum_p alpha(p) (pixel alphas from the C oracle's
    projection record)."""
    Y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    sc = dict(means=np.array([[0.0, 0.0, 3.0]], np.float32),
              scales=np.full((1, 3), 0.15, np.float32),
              quats=np.array([[1.0, 0.0, 0.0, 0.0]], np.float32),
              opacity=np.array([0.6], np.float32),
              sh=np.array([[[0.3, -0.2, 0.1]]], np.float32), sh_degree=0)
    W, H, intr = 24, 20, np.array([30.0, 30.0, 12.0, 10.0], np.float32)
    gr = np.zeros((1, H, W, 3))
    gr[..., 0] = 1.0
    g = B.grads(sc, IDENT_POSE[None], intr[None], W, H, gr)
    rec = oracle.project_all(sc, IDENT_POSE, intr, W, H)
    jj, ii = np.mgrid[0:H, 0:W]
    dx, dy = ii + 0.5 - rec["u"][0], jj + 0.5 - rec["v"][0]
    q = rec["conic_a"][0] * dx * dx + 2 * rec["conic_b"][0] * dx * dy + rec["conic_c"][0] * dy * dy
    a = float(sc["opacity"][0]) * np.exp(-q / 2)
    a = np.where(a >= B.ALPHA_MIN, a, 0.0)
    assert a.max() < B.ALPHA_MAX
    c_r = float(sc["sh"][0, 0, 0]) * Y00 + 0.5
    assert g["opacity"][0] == pytest.approx(c_r * a.sum() / float(sc["opacity"][0]), rel=1e-10)
    assert g["sh"][0, 0, 0] == pytest.approx(Y00 * a.sum(), rel=1e-10)
    assert g["sh"][0, 0, 1] == 0.0 and g["sh"][0, 0, 2] == 0.0
    # symmetric about the optical axis with a symmetric upstream: no sideways pull
    # (the principal point sits on a pixel corner, so the image is symmetric)
    assert abs(g["means"][0, 0]) < 1e-10 and abs(g["means"][0, 1]) < 1e-10


def test_gaussians_out_of_view_get_no_gradient():
    sc = scenegen.tiny_scene(6, 5, sh_degree=1, spread=0.3)
    sc["means"][2] = (0.3, 0.2, -3.0)      # behind the camera
    sc["means"][4] = (40.0, 0.0, 3.0)      # far outside the image
    W, H = 16, 12
    gr, gd, ga = _upstream(1, W, H, 7)
    g = B.grads(sc, IDENT_POSE[None], np.array([[15, 15, 8, 6]], np.float32), W, H, gr, gd, ga)
    for k in ("means", "scales", "quats", "opacity", "sh"):
        assert np.all(g[k][2] == 0) and np.all(g[k][4] == 0), k
        assert np.any(g[k][0] != 0), k
