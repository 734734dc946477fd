"""Pins of the FP64 oracle against facts that do not come from the oracle.

The paper renders with 3D Gaussian splatting (Sec. 3.2) and gets depth from
the same rasterisation (Fig. "Rendering RGB and Depth"); it prints no worked
example, so the pins are closed forms, library routines, finite differences,
Monte Carlo and explicit product formulas:

* quaternion rotation          -> scipy.spatial.transform.Rotation
* real SH basis (CS phase)     -> scipy.special.sph_harm_y, quadrature orthonormality
* EWA 2D covariance            -> closed form on the optical axis, finite-difference
                                  Jacobian of the pinhole map, Monte Carlo
* single-Gaussian image        -> closed form in mpmath (50 digits)
* compositing rules            -> two/three-Gaussian closed forms, stop/skip cases
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle

mp.mp.dps = 50
F32 = lambda x: float(np.float32(x))  # noqa: E731
AMAX, AMIN, TMIN, LOWPASS = F32(0.99), F32(1 / 255), F32(1e-4), F32(0.3)
Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def scene_of(means, scales, quats, opac, rgb):
    """SH-degree-0 scene whose colour is rgb (DC = (rgb - 0.5) / Y00)."""
    means = np.atleast_2d(np.asarray(means, np.float64))
    n = len(means)
    sh = ((np.atleast_2d(rgb) - 0.5) / Y00).astype(np.float32).reshape(n, 1, 3)
    return dict(means=means.astype(np.float32), scales=np.atleast_2d(scales).astype(np.float32),
                quats=np.atleast_2d(quats).astype(np.float32),
                opacity=np.atleast_1d(opac).astype(np.float32), sh=sh, sh_degree=0)


def colour_of(scene, g):
    """Degree-0 colour exactly as stored (the FP32 coefficient times Y00)."""
    return [max(0.0, float(scene["sh"][g, 0, c]) * Y00 + 0.5) for c in range(3)]


IDENT_POSE = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)


# ------------------------------------------------------------ rotations ----

def test_quaternion_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(50):
        q = rng.normal(size=4) * rng.uniform(0.1, 3.0)
        R = oracle.quat_to_rot(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        np.testing.assert_allclose(R, ref, atol=1e-12)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1.0) < 1e-12


# ------------------------------------------------------ spherical harmonics ----

def real_sh_scipy(l, m, d):
    """Real SH with the Condon-Shortley phase kept, from scipy's complex
    Y_l^m (which includes the phase): sqrt2 Re Y_l^m for m > 0,
    sqrt2 Im Y_l^|m| for m < 0, Y_l^0 for m = 0."""
    d = np.asarray(d, np.float64) / np.linalg.norm(d)
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0])
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2) * y.real
    if m < 0:
        return math.sqrt(2) * y.imag
    return y.real


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(2)
    for _ in range(40):
        d = rng.normal(size=3)
        for l in range(4):
            for m in range(-l, l + 1):
                assert oracle.sh_basis(l, m, d) == pytest.approx(real_sh_scipy(l, m, d), abs=1e-12)


def test_sh_basis_low_order_signs():
    # The Condon-Shortley phase makes the l = 1 functions -c y, c z, -c x.
    c = math.sqrt(3 / (4 * math.pi))
    d = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    assert oracle.sh_basis(1, -1, d) == pytest.approx(-c * d[1], abs=1e-14)
    assert oracle.sh_basis(1, 0, d) == pytest.approx(c * d[2], abs=1e-14)
    assert oracle.sh_basis(1, 1, d) == pytest.approx(-c * d[0], abs=1e-14)


def test_sh_basis_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x trapezoid in phi integrates products of
    # degree <= 6 polynomials on the sphere exactly.
    xs, ws = np.polynomial.legendre.leggauss(16)
    phis = np.linspace(0, 2 * np.pi, 32, endpoint=False)
    dirs, wts = [], []
    for x, w in zip(xs, ws):
        s = math.sqrt(1 - x * x)
        for p in phis:
            dirs.append((s * math.cos(p), s * math.sin(p), x))
            wts.append(w * 2 * np.pi / len(phis))
    idx = [(l, m) for l in range(4) for m in range(-l, l + 1)]
    Y = np.array([[oracle.sh_basis(l, m, d) for d in dirs] for (l, m) in idx])
    G = (Y * np.array(wts)) @ Y.T
    np.testing.assert_allclose(G, np.eye(16), atol=1e-10)


def test_sh_colour_degree0_is_rgb_and_clamped():
    rgb = np.array([0.2, 0.7, 1.3])
    coef = ((rgb - 0.5) / Y00).reshape(1, 3)
    out = oracle.sh_color(0, [0.1, 0.2, 0.9], coef)
    np.testing.assert_allclose(out, rgb, atol=1e-14)   # no upper clamp
    out = oracle.sh_color(0, [0.1, 0.2, 0.9], np.array([[-10.0, 0.0, 0.0]]))
    assert out[0] == 0.0 and out[1] == pytest.approx(0.5)


def test_sh_colour_uses_camera_to_mean_direction():
    # A pure l=1, m=0 (z) coefficient: colour = 0.5 + k * c * d_z where d is
    # the unit direction from the camera centre to the mean in world space.
    k = 0.3
    sh = np.zeros((1, 16, 3), np.float32)
    sh[0, 2, :] = k
    mean = np.array([[0.4, -0.2, 3.0]], np.float32)
    sc = dict(means=mean, scales=np.full((1, 3), 0.05, np.float32),
              quats=np.array([[1, 0, 0, 0]], np.float32), opacity=np.array([0.5], np.float32),
              sh=sh, sh_degree=3)
    C = np.array([0.1, 0.3, -1.0], np.float32).astype(np.float64)   # as the FP32 pose holds it
    pose = np.concatenate([np.eye(3), C[:, None]], axis=1)
    rec = oracle.project_all(sc, pose, [50, 50, 32, 24], 64, 48)
    d = mean[0].astype(np.float64) - C
    d /= np.linalg.norm(d)
    expect = 0.5 + float(np.float32(k)) * math.sqrt(3 / (4 * math.pi)) * d[2]
    assert rec["r"][0] == pytest.approx(expect, abs=1e-12)


# ------------------------------------------------------------ projection ----

def test_ewa_on_axis_closed_form():
    fx, fy, z0 = 60.0, 45.0, 3.0
    sx, sy, sz = 0.05, 0.02, 0.03
    sc = scene_of([0, 0, z0], [sx, sy, sz], [1, 0, 0, 0], 0.8, [0.5, 0.5, 0.5])
    rec = oracle.project_all(sc, IDENT_POSE, [fx, fy, 32, 24], 64, 48)
    sxf, syf = F32(sx), F32(sy)
    assert rec["cov_a"][0] == pytest.approx((fx * sxf / z0) ** 2 + LOWPASS, rel=1e-12)
    assert rec["cov_c"][0] == pytest.approx((fy * syf / z0) ** 2 + LOWPASS, rel=1e-12)
    assert abs(rec["cov_b"][0]) < 1e-14
    assert rec["u"][0] == pytest.approx(32.0) and rec["v"][0] == pytest.approx(24.0)
    assert rec["z"][0] == pytest.approx(z0)


def pinhole_jacobian_fd(p, fx, fy, h=mp.mpf("1e-20")):
    """Central finite-difference Jacobian of (fx x/z, fy y/z) in mpmath."""
    def pi(q):
        return [fx * q[0] / q[2], fy * q[1] / q[2]]
    J = mp.matrix(2, 3)
    for j in range(3):
        a = [mp.mpf(v) for v in p]
        b = [mp.mpf(v) for v in p]
        a[j] += h
        b[j] -= h
        fa, fb = pi(a), pi(b)
        for i in range(2):
            J[i, j] = (fa[i] - fb[i]) / (2 * h)
    return J


def rot_world_cov(q, s):
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    return R @ np.diag(np.asarray(s, np.float64) ** 2) @ R.T


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ewa_matches_finite_difference_jacobian(seed):
    rng = np.random.default_rng(seed + 10)
    fx, fy, cx, cy, W, H = 50.0, 55.0, 32.0, 24.0, 64, 48
    mean = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.6, 0.6), rng.uniform(2, 4)])
    q = rng.normal(size=4)
    s = np.exp(rng.normal(-3, 0.3, size=3))
    sc = scene_of(mean, s, q, 0.7, [0.5, 0.5, 0.5])
    # camera rotated about y and translated; world mean = C + R_cw p_cam
    Rcw = Rotation.from_euler("y", 20, degrees=True).as_matrix()
    C = np.array([0.5, -0.2, 1.0])
    mean_w = (C + Rcw @ mean).astype(np.float32)
    sc["means"] = mean_w[None, :]
    pose = np.concatenate([Rcw, C[:, None]], axis=1).astype(np.float32)
    rec = oracle.project_all(sc, pose, [fx, fy, cx, cy], W, H)
    # camera-frame mean from the FP32 inputs, in FP64
    Rcw64 = pose[:, :3].astype(np.float64)
    p = Rcw64.T @ (mean_w.astype(np.float64) - pose[:, 3].astype(np.float64))
    assert abs(p[0] / p[2]) < 1.3 * cx / fx and abs(p[1] / p[2]) < 1.3 * cy / fy
    J = np.array(pinhole_jacobian_fd(p, fx, fy).tolist(), dtype=np.float64)
    Sig_w = rot_world_cov(sc["quats"][0].astype(np.float64), sc["scales"][0].astype(np.float64))
    Sig_c = Rcw64.T @ Sig_w @ Rcw64
    cov = J @ Sig_c @ J.T + LOWPASS * np.eye(2)
    np.testing.assert_allclose([rec["cov_a"][0], rec["cov_b"][0], rec["cov_c"][0]],
                               [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-9, atol=1e-12)
    assert rec["u"][0] == pytest.approx(fx * p[0] / p[2] + cx, rel=1e-12)
    assert rec["v"][0] == pytest.approx(fy * p[1] / p[2] + cy, rel=1e-12)
    inv = np.linalg.inv(cov)
    np.testing.assert_allclose([rec["conic_a"][0], rec["conic_b"][0], rec["conic_c"][0]],
                               [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-9)


def test_ewa_monte_carlo():
    # A small Gaussian: the covariance of exactly projected samples tends to
    # the first-order (EWA) covariance J Sigma J^T.
    rng = np.random.default_rng(5)
    mean = np.array([0.3, -0.2, 3.0])
    q = np.array([0.9, 0.2, -0.3, 0.1])
    s = np.array([0.01, 0.004, 0.007])
    sc = scene_of(mean, s, q, 0.7, [0.5, 0.5, 0.5])
    fx = fy = 400.0
    rec = oracle.project_all(sc, IDENT_POSE, [fx, fy, 320, 240], 640, 480)
    Sig = rot_world_cov(sc["quats"][0].astype(np.float64), sc["scales"][0].astype(np.float64))
    X = rng.multivariate_normal(sc["means"][0].astype(np.float64), Sig, size=400_000)
    uv = np.stack([fx * X[:, 0] / X[:, 2], fy * X[:, 1] / X[:, 2]], axis=1)
    emp = np.cov(uv.T)
    got = np.array([[rec["cov_a"][0] - LOWPASS, rec["cov_b"][0]],
                    [rec["cov_b"][0], rec["cov_c"][0] - LOWPASS]])
    np.testing.assert_allclose(emp, got, rtol=0.02, atol=0.02 * got[0, 0])


def test_near_plane_and_zero_opacity_are_inert():
    base = scene_of([[0, 0, 3.0]], [[0.05, 0.05, 0.05]], [[1, 0, 0, 0]], [0.6], [[0.9, 0.1, 0.3]])
    extra = scene_of([[0.0, 0.0, 0.15], [0.05, 0.0, 2.0]], [[0.1] * 3, [0.2] * 3],
                     [[1, 0, 0, 0]] * 2, [0.9, F32(1 / 255) * 0.99], [[1, 1, 1], [1, 0, 0]])
    both = {k: np.concatenate([base[k], extra[k]]) if k != "sh_degree" else 0 for k in base}
    intr = [50, 50, 32, 24]
    a = oracle.render(base, IDENT_POSE, intr, 64, 48)
    b = oracle.render(both, IDENT_POSE, intr, 64, 48)
    np.testing.assert_array_equal(a.rgb, b.rgb)
    np.testing.assert_array_equal(a.depth, b.depth)


# -------------------------------------------------------- single Gaussian ----

def closed_form_image(u, v, cov, o, rgb, z, W, H):
    """alpha(p) = min(0.99, o exp(-1/2 d^T cov^-1 d)); pixel = alpha rgb,
    depth z, alpha alpha where alpha >= 1/255, else 0 (mpmath)."""
    a, b, c = (mp.mpf(x) for x in cov)
    det = a * c - b * b
    out = np.zeros((H, W, 5))
    margin = np.zeros((H, W))
    for j in range(H):
        for i in range(W):
            dx = mp.mpf(i) + mp.mpf("0.5") - mp.mpf(u)
            dy = mp.mpf(j) + mp.mpf("0.5") - mp.mpf(v)
            q = (c * dx * dx - 2 * b * dx * dy + a * dy * dy) / det
            al = min(mp.mpf(AMAX), mp.mpf(o) * mp.exp(-q / 2))
            margin[j, i] = float(abs(al - AMIN) / AMIN)
            if al >= AMIN:
                out[j, i, :3] = [float(al * mp.mpf(x)) for x in rgb]
                out[j, i, 3] = z
                out[j, i, 4] = float(al)
    return out, margin


def check_single(sc, intr, W, H, cov):
    r = oracle.render(sc, IDENT_POSE, intr, W, H)
    rec = oracle.project_all(sc, IDENT_POSE, intr, W, H)
    img, margin = closed_form_image(rec["u"][0], rec["v"][0], cov, float(sc["opacity"][0]),
                                    colour_of(sc, 0), float(sc["means"][0, 2]), W, H)
    safe = margin > 1e-9
    np.testing.assert_allclose(r.rgb[safe], img[..., :3][safe], atol=1e-13)
    np.testing.assert_allclose(r.depth[safe], img[..., 3][safe], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r.alpha[safe], img[..., 4][safe], atol=1e-13)
    # the footprint cutoff runs through the image: both sides are present
    assert (img[..., 4] > 0).sum() > 10 and (img[..., 4] == 0).sum() > 10
    return r, img


def test_single_gaussian_isotropic_on_axis():
    fx, z0, s = 50.0, 3.0, 0.15
    sc = scene_of([0, 0, z0], [s, s, s], [1, 0, 0, 0], 0.7, [0.9, 0.4, 0.1])
    sf = F32(s)
    var = (fx * sf / z0) ** 2 + LOWPASS
    check_single(sc, [fx, fx, 32.0, 24.0], 64, 48, (var, 0.0, var))


def test_single_gaussian_rotated_90_swaps_axes():
    fx, z0, sx, sy = 50.0, 3.0, 0.3, 0.08
    h = math.sqrt(0.5)
    sc = scene_of([0, 0, z0], [sx, sy, 0.1], [h, 0, 0, h], 0.9, [0.2, 0.8, 0.5])
    var_x = (fx * F32(sy) / z0) ** 2 + LOWPASS
    var_y = (fx * F32(sx) / z0) ** 2 + LOWPASS
    check_single(sc, [fx, fx, 32.0, 24.0], 64, 48, (var_x, 0.0, var_y))


def test_single_gaussian_rotated_45_off_diagonal_sign():
    fx, z0, sx, sy = 50.0, 3.0, 0.3, 0.08
    c, s = math.cos(math.pi / 8), math.sin(math.pi / 8)
    sc = scene_of([0, 0, z0], [sx, sy, 0.1], [c, 0, 0, s], 0.9, [0.2, 0.8, 0.5])
    q = sc["quats"][0].astype(np.float64)
    Sig = rot_world_cov(q, sc["scales"][0].astype(np.float64))
    k = (fx / z0) ** 2
    cov = (k * Sig[0, 0] + LOWPASS, k * Sig[0, 1], k * Sig[1, 1] + LOWPASS)
    assert cov[1] > 0   # +45 deg: elongated along x = y
    r, img = check_single(sc, [fx, fx, 32.0, 24.0], 64, 48, cov)
    # mirror check: pixel (32+6, 24+6) is brighter than (32+6, 24-6)
    assert r.alpha[30, 38] > r.alpha[18, 38]


def test_single_gaussian_off_axis_fd_jacobian():
    fx, fy = 50.0, 50.0
    mean = np.array([0.5, -0.3, 3.0])
    s = 0.12
    sc = scene_of(mean, [s, s, s], [1, 0, 0, 0], 0.8, [0.6, 0.6, 0.2])
    p = sc["means"][0].astype(np.float64)
    J = np.array(pinhole_jacobian_fd(p, fx, fy).tolist(), dtype=np.float64)
    cov = J @ (np.eye(3) * F32(s) ** 2) @ J.T + LOWPASS * np.eye(2)
    check_single(sc, [fx, fy, 32.0, 24.0], 64, 48, (cov[0, 0], cov[0, 1], cov[1, 1]))


def test_single_gaussian_opaque_centre_clamped():
    fx, z0, s = 50.0, 3.0, 0.2
    sc = scene_of([0, 0, z0], [s, s, s], [1, 0, 0, 0], 1.0, [1.0, 0.5, 0.25])
    intr = [fx, fx, 32.5, 24.5]   # the mean projects onto pixel centre (32, 24)
    r = oracle.render(sc, IDENT_POSE, intr, 64, 48)
    assert r.alpha[24, 32] == AMAX
    np.testing.assert_allclose(r.rgb[24, 32], np.array(colour_of(sc, 0)) * AMAX, atol=1e-15)


def test_below_cutoff_contributes_nothing():
    o = AMIN * 0.999
    sc = scene_of([0, 0, 3.0], [0.3] * 3, [1, 0, 0, 0], o, [1, 1, 1])
    r = oracle.render(sc, IDENT_POSE, [50, 50, 32.5, 24.5], 64, 48)
    assert np.all(r.rgb == 0) and np.all(r.depth == 0) and np.all(r.alpha == 0)


# ------------------------------------------------------------- compositing ----

def test_two_and_three_gaussians_closed_form():
    fx = 50.0
    zs = [2.0, 3.0, 4.5]
    ss = [0.08, 0.15, 0.3]
    os_ = [0.6, 0.7, 0.8]
    cols = [[0.9, 0.1, 0.1], [0.1, 0.9, 0.1], [0.1, 0.1, 0.9]]
    for n in (2, 3):
        sc = scene_of([[0, 0, z] for z in zs[:n]], [[s] * 3 for s in ss[:n]],
                      [[1, 0, 0, 0]] * n, os_[:n], cols[:n])
        intr = [fx, fx, 32.0, 24.0]
        r = oracle.render(sc, IDENT_POSE, intr, 64, 48)
        for (j, i) in [(24, 32), (26, 35), (20, 28), (24, 38), (24, 40)]:
            dx, dy = i + 0.5 - 32.0, j + 0.5 - 24.0
            T = mp.mpf(1)
            acc = [mp.mpf(0)] * 5
            for g in range(n):
                var = (fx * F32(ss[g]) / zs[g]) ** 2 + LOWPASS
                al = min(mp.mpf(AMAX), mp.mpf(F32(os_[g])) * mp.exp(-(dx * dx + dy * dy) / (2 * var)))
                if al < AMIN:
                    continue
                assert T * (1 - al) >= TMIN
                c = colour_of(sc, g)
                for ch in range(3):
                    acc[ch] += al * T * c[ch]
                acc[3] += al * T * zs[g]
                acc[4] += al * T
                T *= (1 - al)
            np.testing.assert_allclose(r.rgb[j, i], [float(x) for x in acc[:3]], atol=1e-13)
            assert r.alpha[j, i] == pytest.approx(float(acc[4]), abs=1e-13)
            if acc[4] > 0:
                assert r.depth[j, i] == pytest.approx(float(acc[3] / acc[4]), rel=1e-13)
            else:
                assert r.depth[j, i] == 0.0
            assert r.tfinal[j, i] == pytest.approx(float(T), rel=1e-12)


def test_two_saturated_gaussians_stop_excludes_second():
    # (1 - fl32(0.99))^2 = 9.99998e-5 < fl32(1e-4): the second Gaussian is
    # not accumulated at the centre pixel.
    sc = scene_of([[0, 0, 2.0], [0, 0, 3.0]], [[0.2] * 3, [0.3] * 3], [[1, 0, 0, 0]] * 2,
                  [1.0, 1.0], [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    r = oracle.render(sc, IDENT_POSE, [50, 50, 32.5, 24.5], 64, 48)
    c1 = colour_of(sc, 0)
    np.testing.assert_allclose(r.rgb[24, 32], np.array(c1) * AMAX, atol=1e-15)
    assert r.depth[24, 32] == pytest.approx(2.0, rel=1e-15)
    assert r.alpha[24, 32] == AMAX
    assert r.tfinal[24, 32] == pytest.approx(1 - AMAX, rel=1e-15)
    # the decision is within rounding of the threshold, so it is flagged
    assert 24 * 64 + 32 in set(r.var_pix.tolist())


def test_stop_after_third_of_four():
    # alpha = 0.95 each: T = 2.5e-3, 1.25e-4 (>= 1e-4, kept), then 6.25e-6
    # (< 1e-4): the fourth Gaussian is not accumulated.
    sc = scene_of([[0, 0, 2.0], [0, 0, 3.0], [0, 0, 4.0], [0, 0, 5.0]], [[0.3] * 3] * 4,
                  [[1, 0, 0, 0]] * 4, [0.95] * 4, [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]])
    r = oracle.render(sc, IDENT_POSE, [50, 50, 32.5, 24.5], 64, 48)
    a = F32(0.95)
    assert r.tfinal[24, 32] == pytest.approx((1 - a) ** 3, rel=1e-12)
    c = [colour_of(sc, g) for g in range(4)]
    expect = [a * c[0][ch] + (1 - a) * a * c[1][ch] + (1 - a) ** 2 * a * c[2][ch]
              for ch in range(3)]
    np.testing.assert_allclose(r.rgb[24, 32], expect, atol=1e-14)
    w = [a, (1 - a) * a, (1 - a) ** 2 * a]
    assert r.depth[24, 32] == pytest.approx((2 * w[0] + 3 * w[1] + 4 * w[2]) / sum(w), rel=1e-13)


# ------------------------------------------------------------ motion blur ----

def test_motion_blur_without_motion_is_the_plain_render():
    sc = scene_of([[0, 0, 3.0], [0.2, -0.1, 3.5]], [[0.15] * 3, [0.2, 0.1, 0.1]],
                  [[1, 0, 0, 0]] * 2, [0.7, 0.9], [[0.9, 0.4, 0.1], [0.1, 0.5, 0.8]])
    intr = [50.0, 50.0, 32.0, 24.0]
    ref = oracle.render(sc, IDENT_POSE, intr, 64, 48)
    rgb, depth, alpha, subs = oracle.render_motion_blur(sc, IDENT_POSE, [0, 0, 0], intr, 64, 48,
                                                        shutter=0.02, n_sub=5)
    assert len(subs) == 5
    np.testing.assert_allclose(rgb, ref.rgb, atol=1e-15)
    np.testing.assert_allclose(depth, ref.depth, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(alpha, ref.alpha, atol=1e-15)


def test_motion_blur_single_gaussian_sideways_closed_form():
    """A camera sliding along its x axis sees one isotropic Gaussian at
    u_k = fx x_k / z + cx with the off-axis EWA covariance
    s^2 fx^2 / z^2 (1 + x_k^2 / z^2) + 0.3 along x and s^2 fy^2 / z^2 + 0.3
    along y: the blurred frame is the mean of those closed-form images, its
    depth z wherever any sub-frame is covered."""
    fx, z0, s, o = 50.0, 3.0, 0.12, 0.8
    sc = scene_of([0, 0, z0], [s, s, s], [1, 0, 0, 0], o, [0.9, 0.4, 0.1])
    vel, shutter, K = np.array([12.0, 0.0, 0.0]), 0.05, 4
    intr = [fx, fx, 32.0, 24.0]
    rgb, depth, alpha, _ = oracle.render_motion_blur(sc, IDENT_POSE, vel, intr, 64, 48,
                                                     shutter=shutter, n_sub=K)
    sf = F32(s)
    imgs, margins = [], []
    for k in range(K):
        dt = np.float32(float(np.float32(shutter)) * (k + 0.5) / K)
        cx_cam = np.float32(0.0) - np.float32(vel[0]) * dt   # camera centre x (FP32 input)
        x = -float(cx_cam)                                    # Gaussian x in the camera frame
        var_x = sf * sf * fx * fx / (z0 * z0) * (1 + x * x / (z0 * z0)) + LOWPASS
        var_y = (fx * sf / z0) ** 2 + LOWPASS
        img, mar = closed_form_image(fx * x / z0 + 32.0, 24.0, (var_x, 0.0, var_y), F32(o),
                                     colour_of(sc, 0), z0, 64, 48)
        imgs.append(img)
        margins.append(mar)
    safe = np.min(margins, axis=0) > 1e-9
    mean = sum(imgs) / K
    np.testing.assert_allclose(rgb[safe], mean[..., :3][safe], atol=1e-12)
    np.testing.assert_allclose(alpha[safe], mean[..., 4][safe], atol=1e-12)
    covered = safe & (mean[..., 4] > 0)
    np.testing.assert_allclose(depth[covered], z0, rtol=1e-12)
    assert np.all(depth[safe & (mean[..., 4] == 0)] == 0)
    # the blur is visible: the covered extent along x exceeds one sub-frame's
    assert (mean[..., 4] > 0).sum() > (imgs[0][..., 4] > 0).sum() + 10


# ---------------------------------------------------------------- golden ----

def test_oracle_matches_stored_workload0_values():
    """The oracle still gives the values stored by
    tests/golden/make_workload0_oracle.py (regression pin of its arithmetic;
    the file is regenerated only with a change justified by the paper)."""
    import os
    import scenegen
    path = os.path.join(os.path.dirname(__file__), "golden", "workload0_oracle.txt")
    rows = [list(map(float, l.split())) for l in open(path) if not l.startswith("#")]
    sc = scenegen.make_scene(0)
    cams = scenegen.make_cameras(0)
    ref = oracle.render(sc, cams["poses"][0], cams["intrinsics"][0], 64, 48)
    assert len(rows) > 50 and sum(r[6] > 0 for r in rows) > 30
    for i, j, r, g, b, d, a in rows:
        i, j = int(i), int(j)
        np.testing.assert_allclose(ref.rgb[j, i], [r, g, b], rtol=1e-12, atol=1e-15)
        assert ref.depth[j, i] == pytest.approx(d, rel=1e-12, abs=1e-15)
        assert ref.alpha[j, i] == pytest.approx(a, rel=1e-12, abs=1e-15)
