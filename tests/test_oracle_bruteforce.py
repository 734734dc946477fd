"""Brute-force, invariant and comparator checks of the FP64 oracle.

The compositing walk of the oracle (front-to-back, skip below 1/255, stop
before T drops under 1e-4) is checked against the explicit product form
C(p) = sum_{i<=k} c_i a_i prod_{j<i} (1 - a_j) evaluated in mpmath over the
(z, index)-ordered candidates, on tiny scenes; then invariants that hold for
any scene (transmittance range, weight sum, colour bound, depth range,
permutation, rigid-motion invariance).
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenegen

mp.mp.dps = 40
F32 = lambda x: float(np.float32(x))  # noqa: E731
AMAX, AMIN, TMIN = F32(0.99), F32(1 / 255), F32(1e-4)
IDENT_POSE = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
TINY_INTR = [8.0, 8.0, 4.0, 4.0]


def product_form(rec, W, H):
    """Explicit product formula per pixel from the per-Gaussian records."""
    n = len(rec["u"])
    out = np.zeros((H, W, 5))
    for j in range(H):
        for i in range(W):
            cands = []
            for g in range(n):
                if not rec["in_front"][g]:
                    continue
                dx = mp.mpf(i) + mp.mpf(0.5) - mp.mpf(rec["u"][g])
                dy = mp.mpf(j) + mp.mpf(0.5) - mp.mpf(rec["v"][g])
                q = (mp.mpf(rec["conic_a"][g]) * dx * dx + 2 * mp.mpf(rec["conic_b"][g]) * dx * dy +
                     mp.mpf(rec["conic_c"][g]) * dy * dy)
                a = min(mp.mpf(AMAX), mp.mpf(rec["opacity"][g]) * mp.exp(-q / 2))
                if a >= AMIN:
                    cands.append((rec["z"][g], g, a))
            cands.sort(key=lambda t: (t[0], t[1]))
            # included prefix: largest k with prod_{j<=k}(1 - a_j) >= T_MIN
            k, prod = 0, mp.mpf(1)
            while k < len(cands) and prod * (1 - cands[k][2]) >= TMIN:
                prod *= 1 - cands[k][2]
                k += 1
            rgbz = [mp.mpf(0)] * 5
            for idx in range(k):
                z, g, a = cands[idx]
                w = a
                for jj in range(idx):
                    w *= 1 - cands[jj][2]
                for ch, key in enumerate(("r", "g", "b")):
                    rgbz[ch] += w * mp.mpf(rec[key][g])
                rgbz[3] += w * mp.mpf(z)
                rgbz[4] += w
            out[j, i, :3] = [float(x) for x in rgbz[:3]]
            out[j, i, 3] = float(rgbz[3] / rgbz[4]) if rgbz[4] > 0 else 0.0
            out[j, i, 4] = float(rgbz[4])
    return out


@pytest.mark.parametrize("seed,n,opac_boost", [(0, 6, 0.0), (1, 8, 0.0), (2, 10, 3.0),
                                                (3, 12, 5.0), (4, 5, -1.0)])
def test_bruteforce_product_form(seed, n, opac_boost):
    if opac_boost >= 3.0:   # dense, nearly opaque cluster: the stop rule fires
        sc = scenegen.tiny_scene(n, seed, sh_degree=(seed % 2) * 3, spread=0.2,
                                 log_scale_mean=-0.8)
    else:
        sc = scenegen.tiny_scene(n, seed, sh_degree=(seed % 2) * 3)
    if opac_boost:
        logit = np.log(sc["opacity"] / (1 - sc["opacity"])) + opac_boost
        sc["opacity"] = (1 / (1 + np.exp(-logit))).astype(np.float32)
    W = H = 8
    r = oracle.render(sc, IDENT_POSE, TINY_INTR, W, H)
    rec = oracle.project_all(sc, IDENT_POSE, TINY_INTR, W, H)
    ref = product_form(rec, W, H)
    flagged = set(r.var_pix.tolist())
    for j in range(H):
        for i in range(W):
            if j * W + i in flagged:
                continue
            np.testing.assert_allclose(r.rgb[j, i], ref[j, i, :3], atol=1e-12)
            assert r.depth[j, i] == pytest.approx(ref[j, i, 3], rel=1e-12, abs=1e-12)
            assert r.alpha[j, i] == pytest.approx(ref[j, i, 4], abs=1e-12)
    assert r.counters["pairs"] > 0
    if opac_boost >= 3.0:
        assert r.tfinal.min() < 1e-3   # the stop rule is exercised


@pytest.mark.parametrize("seed", [0, 1])
def test_permutation_invariance(seed):
    sc = scenegen.tiny_scene(40, seed + 100, sh_degree=3)
    perm = np.random.default_rng(seed).permutation(40)
    sp = {k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    a = oracle.render(sc, IDENT_POSE, [20, 20, 16, 12], 32, 24)
    b = oracle.render(sp, IDENT_POSE, [20, 20, 16, 12], 32, 24)
    np.testing.assert_array_equal(a.rgb, b.rgb)
    np.testing.assert_array_equal(a.depth, b.depth)


def _workload0_render():
    sc = scenegen.make_scene(0)
    cams = scenegen.make_cameras(0)
    return sc, cams, oracle.render(sc, cams["poses"][0], cams["intrinsics"][0], 64, 48)


def test_invariants_workload0():
    sc, cams, r = _workload0_render()
    assert r.tfinal.min() >= TMIN and r.tfinal.max() <= 1.0
    np.testing.assert_allclose(r.alpha, 1.0 - r.tfinal, atol=1e-12)
    assert r.alpha.max() <= 1.0 - TMIN + 1e-12
    rec = oracle.project_all(sc, cams["poses"][0], cams["intrinsics"][0], 64, 48)
    vis = rec["visible"] > 0
    cmax = max(rec["r"][vis].max(), rec["g"][vis].max(), rec["b"][vis].max())
    assert np.all(r.rgb <= cmax * r.alpha[..., None] + 1e-12)
    has = r.alpha > 0
    assert r.depth[has].min() >= rec["z"][vis].min() - 1e-12
    assert r.depth[has].max() <= rec["z"][vis].max() + 1e-12
    assert np.all(r.depth[~has] == 0)
    assert r.counters["unresolved"] == 0


def _unflagged(*renders):
    H, W = renders[0].depth.shape
    m = np.ones(H * W, bool)
    for r in renders:
        m[r.var_pix] = False
    return m.reshape(H, W)


def test_rigid_motion_invariance():
    sc, cams, a = _workload0_render()
    R = Rotation.from_euler("xyz", [20, -35, 50], degrees=True)
    t = np.array([1.5, -2.0, 0.75])
    sc2 = dict(sc)
    sc2["means"] = (R.apply(sc["means"].astype(np.float64)) + t).astype(np.float32)
    q = sc["quats"].astype(np.float64)
    qr = (R * Rotation.from_quat(q[:, [1, 2, 3, 0]])).as_quat()
    sc2["quats"] = qr[:, [3, 0, 1, 2]].astype(np.float32)
    pose = cams["poses"][0].astype(np.float64)
    pose2 = np.concatenate([R.as_matrix() @ pose[:, :3], (R.apply(pose[:, 3]) + t)[:, None]], axis=1)
    b = oracle.render(sc2, pose2.astype(np.float32), cams["intrinsics"][0], 64, 48)
    m = _unflagged(a, b)
    np.testing.assert_allclose(b.rgb[m], a.rgb[m], atol=1e-4)
    np.testing.assert_allclose(b.alpha[m], a.alpha[m], atol=1e-4)
    np.testing.assert_allclose(b.depth[m], a.depth[m], rtol=1e-5, atol=1e-6)


# ------------------------------------------------------------- comparator ----

def test_comparator_accepts_itself_and_rejects_planted_errors():
    sc, cams, r = _workload0_render()
    rep = oracle.compare(r, r.rgb, r.depth, r.alpha)
    assert rep["failed"] == 0 and rep["max_abs_rgb"] == 0.0
    rgb = r.rgb.copy()
    rgb[10, 20, 1] += 3e-3
    assert oracle.compare(r, rgb, r.depth, r.alpha)["failed"] == 1
    dep = r.depth.copy()
    j, i = np.argwhere(r.alpha > 0.5)[0]
    dep[j, i] *= 1.002
    assert oracle.compare(r, r.rgb, dep, r.alpha)["failed"] == 1
    dep = r.depth.copy()
    j, i = np.argwhere(r.alpha == 0)[0] if (r.alpha == 0).any() else (0, 0)
    if r.alpha[j, i] == 0:
        dep[j, i] = 0.5
        assert oracle.compare(r, r.rgb, dep, r.alpha)["failed"] == 1


def test_comparator_rescues_listed_alternatives():
    sc, cams, r = _workload0_render()
    assert len(r.var_pix) > 0
    # replace every flagged pixel by its last listed alternative
    rgb, dep, alp = r.rgb.copy(), r.depth.copy(), r.alpha.copy()
    W = r.depth.shape[1]
    changed = 0
    for p in np.unique(r.var_pix):
        rows = r.var_vals[r.var_pix == p]
        v = rows[-1]
        j, i = divmod(int(p), W)
        if np.max(np.abs(v[:3] - rgb[j, i])) > 2e-3:
            changed += 1
        rgb[j, i], dep[j, i], alp[j, i] = v[:3], v[3], v[4]
    rep = oracle.compare(r, rgb, dep, alp)
    assert rep["failed"] == 0
    assert rep["rescued"] >= changed
    # an image without an alpha channel is held to RGB and depth only: the
    # alternatives still rescue it (their weights differ from the FP64 one)
    rep = oracle.compare(r, rgb, dep)
    assert rep["failed"] == 0 and rep["rescued"] >= changed
    assert rep["max_abs_alpha"] == 0.0
    rgb[np.unravel_index(int(r.var_pix[0]), r.depth.shape)] += 0.1
    assert oracle.compare(r, rgb, dep)["failed"] == 1


def test_two_saturated_alternative_is_listed():
    # The second of two alpha = 0.99 Gaussians sits within rounding of the
    # stop threshold: a renderer that includes it is also accepted.
    Y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    cols = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    sc = dict(means=np.array([[0, 0, 2.0], [0, 0, 3.0]], np.float32),
              scales=np.full((2, 3), 0.25, np.float32),
              quats=np.tile(np.array([1, 0, 0, 0], np.float32), (2, 1)),
              opacity=np.ones(2, np.float32),
              sh=((cols - 0.5) / Y00).astype(np.float32).reshape(2, 1, 3), sh_degree=0)
    r = oracle.render(sc, IDENT_POSE, [50, 50, 32.5, 24.5], 64, 48)
    rgb = r.rgb.copy()
    c1 = float(sc["sh"][0, 0, 0]) * Y00 + 0.5
    c2 = float(sc["sh"][1, 0, 1]) * Y00 + 0.5
    rgb[24, 32, 1] += (1 - AMAX) * AMAX * c2
    alp = r.alpha.copy()
    alp[24, 32] += (1 - AMAX) * AMAX
    dep = r.depth.copy()
    dep[24, 32] = (AMAX * 2.0 + (1 - AMAX) * AMAX * 3.0) / alp[24, 32]
    assert c1 > 0.99
    rep = oracle.compare(r, rgb, dep, alp)
    assert rep["failed"] == 0 and rep["rescued"] >= 1


def test_near_tie_before_stop_listed_despite_ties_after_stop():
    # Two contributors one FP32 ulp apart in depth early in the walk, then
    # opaque Gaussians that stop it, then many tied pairs past the stop. The
    # swapped order of the first pair must be listed as an alternative.
    Y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    z1 = 2.0
    z2 = float(np.nextafter(np.float32(2.0), np.float32(3.0)))
    zs = [z1, z2, 3.0, 3.1, 3.2]
    zs += [z for k in range(8) for z in (5.0 + k, float(np.nextafter(np.float32(5.0 + k),
                                                                      np.float32(99))))]
    n = len(zs)
    cols = np.full((n, 3), 0.5)
    cols[0] = (1.0, 0.0, 0.0)
    cols[1] = (0.0, 0.0, 1.0)
    op = np.full(n, 0.999, np.float32)
    op[0], op[1] = 0.5, 0.6
    sc = dict(means=np.array([[0.0, 0.0, z] for z in zs], np.float32),
              scales=np.full((n, 3), 0.3, np.float32),
              quats=np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)), opacity=op,
              sh=((cols - 0.5) / Y00).astype(np.float32).reshape(n, 1, 3), sh_degree=0)
    r = oracle.render(sc, IDENT_POSE, [50, 50, 32.5, 24.5], 64, 48)
    p = 24 * 64 + 32
    rows = r.var_vals[r.var_pix == p]
    assert len(rows) >= 2
    # one alternative puts the blue Gaussian first: more blue than the primary
    assert any(v[2] - r.rgb[24, 32, 2] > 1e-2 for v in rows)


def _walk_in_order(rec, order, W, H):
    """Per-pixel walk (skip, stop, accumulate) over the Gaussians in a given
    order, FP64, from the projection records."""
    out = np.zeros((H, W, 5))
    for j in range(H):
        for i in range(W):
            T, acc = 1.0, np.zeros(5)
            for g in order:
                dx, dy = i + 0.5 - rec["u"][g], j + 0.5 - rec["v"][g]
                q = rec["conic_a"][g] * dx * dx + 2 * rec["conic_b"][g] * dx * dy + \
                    rec["conic_c"][g] * dy * dy
                a = min(AMAX, rec["opacity"][g] * math.exp(-q / 2))
                if a < AMIN:
                    continue
                if T * (1 - a) < TMIN:
                    break
                w = a * T
                acc += w * np.array([rec["r"][g], rec["g"][g], rec["b"][g], rec["z"][g], 1.0])
                T *= 1 - a
            out[j, i, :3] = acc[:3]
            out[j, i, 3] = acc[3] / acc[4] if acc[4] > 0 else 0.0
            out[j, i, 4] = acc[4]
    return out


def _tied_scene(k):
    """k Gaussians at exactly the same depth in front of the camera, slightly
    offset sideways, with distinct colours."""
    Y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    rng = np.random.default_rng(70 + k)
    cols = rng.uniform(0, 1, size=(k, 3))
    means = np.array([[0.02 * g, -0.015 * g, 3.0] for g in range(k)], np.float32)
    return dict(means=means, scales=np.full((k, 3), 0.2, np.float32),
                quats=np.tile(np.array([1, 0, 0, 0], np.float32), (k, 1)),
                opacity=np.full(k, 0.45, np.float32),
                sh=((cols - 0.5) / Y00).astype(np.float32).reshape(k, 1, 3), sh_degree=0)


def test_every_order_of_a_tied_run_is_accepted():
    """Three contributors at exactly the same depth: the oracle walks them in
    index order, and the comparator accepts an image composited in any of the
    six orders (full reversal included)."""
    import itertools
    sc = _tied_scene(3)
    W, H, intr = 16, 12, [20.0, 20.0, 8.0, 6.0]
    r = oracle.render(sc, IDENT_POSE, intr, W, H)
    rec = oracle.project_all(sc, IDENT_POSE, intr, W, H)
    assert r.counters["unresolved"] == 0
    for perm in itertools.permutations(range(3)):
        img = _walk_in_order(rec, list(perm), W, H)
        rep = oracle.compare(r, img[..., :3], img[..., 3], img[..., 4])
        assert rep["failed"] == 0, (perm, rep)
        if perm != (0, 1, 2):
            assert rep["rescued"] > 0, perm
    # a wrong colour at a tied pixel is still rejected
    img = _walk_in_order(rec, [2, 1, 0], W, H)
    img[6, 8, 0] += 0.05
    assert oracle.compare(r, img[..., :3], img[..., 3], img[..., 4])["failed"] == 1


def test_tied_run_beyond_the_bound_is_unresolved():
    """Five contributors tied in depth exceed the four-member bound: those
    pixels are counted as unresolved and marked by one entry of NaNs (they
    have alternatives the oracle does not list), so the comparator does not
    hold them to the plain-pixel bar, and accepts there only the oracle's
    own order (another order is not confirmed)."""
    sc = _tied_scene(5)
    W, H, intr = 16, 12, [20.0, 20.0, 8.0, 6.0]
    r = oracle.render(sc, IDENT_POSE, intr, W, H)
    n_un = r.counters["unresolved"]
    assert n_un > 0
    marked = np.unique(r.var_pix[np.isnan(r.var_vals).all(axis=1)])
    assert len(marked) == n_un
    rep = oracle.compare(r, r.rgb, r.depth, r.alpha)
    assert rep["failed"] == 0 and rep["unresolved"] == n_un
    assert rep["with_alternatives"] >= n_un
    rec = oracle.project_all(sc, IDENT_POSE, intr, W, H)
    img = _walk_in_order(rec, [4, 3, 2, 1, 0], W, H)
    rep = oracle.compare(r, img[..., :3], img[..., 3], img[..., 4])
    assert 0 < rep["failed"] <= n_un
    assert set(rep["failed_pixels"]) <= set(marked.tolist())   # the first 20 listed
    assert rep["plain_max_abs_rgb"] < 1e-9


# ----------------------------------------------------------- counters ----

def _ellipse_boxes(rec, k=4096):
    """Bounding boxes of the alpha >= 1/255 ellipses, from points sampled on
    each ellipse's boundary (delta = r L (cos t, sin t), Sigma' = L L^T,
    r^2 = 2 ln(o / alpha_min)); NaN where opacity < alpha_min."""
    t = np.linspace(0.0, 2.0 * np.pi, k, endpoint=False)
    out = np.full((len(rec["u"]), 4), np.nan)
    for g in range(len(rec["u"])):
        o = rec["opacity"][g]
        if not rec["in_front"][g] or o < AMIN:
            continue
        S = np.array([[rec["cov_a"][g], rec["cov_b"][g]], [rec["cov_b"][g], rec["cov_c"][g]]])
        L = np.linalg.cholesky(S)
        r = math.sqrt(2.0 * math.log(o / AMIN))
        pts = r * (L @ np.stack([np.cos(t), np.sin(t)]))
        out[g] = (rec["u"][g] + pts[0].min(), rec["u"][g] + pts[0].max(),
                  rec["v"][g] + pts[1].min(), rec["v"][g] + pts[1].max())
    return out


@pytest.mark.parametrize("seed,n,W,H,spread", [(21, 30, 40, 24, 0.9), (22, 60, 48, 40, 0.9),
                                               (23, 15, 33, 17, 0.9), (24, 80, 40, 30, 4.0)])
def test_counters_match_brute_force(seed, n, W, H, spread):
    """The oracle's counters (visible Gaussians, 16x16-tile instances of their
    exact boxes, contributing pairs), against counts taken independently:
    boxes from points sampled on each alpha = 1/255 ellipse, and the
    contributors of every pixel from the product form's included prefix
    (a per-pixel loop in Python floats over the projection records)."""
    sc = scenegen.tiny_scene(n, seed, sh_degree=1, spread=spread, log_scale_mean=-2.0)
    intr = [W * 0.7, W * 0.7, W / 2 + 0.25, H / 2 - 0.35]
    r = oracle.render(sc, IDENT_POSE, intr, W, H)
    rec = oracle.project_all(sc, IDENT_POSE, intr, W, H)
    boxes = _ellipse_boxes(rec)
    vis = tiles = 0
    edge = 0
    for b in boxes:
        if np.isnan(b[0]):
            continue
        # pixel centres i + 1/2 inside [x0, x1], clipped to the image
        x0 = max(0, math.ceil(b[0] - 0.5)); x1 = min(W - 1, math.floor(b[1] - 0.5))
        y0 = max(0, math.ceil(b[2] - 0.5)); y1 = min(H - 1, math.floor(b[3] - 0.5))
        # a box edge within sampling error of a pixel centre may go either way
        if min(abs((b[j] - 0.5) - round(b[j] - 0.5)) for j in range(4)) < 1e-5:
            edge += 1
        if x0 <= x1 and y0 <= y1:
            vis += 1
            tiles += (x1 // 16 - x0 // 16 + 1) * (y1 // 16 - y0 // 16 + 1)
    c = r.counters
    print(f"visible {c['visible']} / {vis}, instances {c['instances16']} / {tiles}, "
          f"edge cases {edge}")
    assert vis > 5
    if spread > 2:
        assert vis < n - 5   # some Gaussians project outside the image
    assert abs(c["visible"] - vis) <= edge
    assert abs(c["instances16"] - tiles) <= 4 * edge
    # contributors per pixel: the included prefix of the product form
    prod = product_form_counts(rec, W, H)
    n_alt = len(np.unique(r.var_pix))
    print(f"pairs {c['pairs']} / {prod}, pixels with alternatives {n_alt}")
    assert abs(c["pairs"] - prod) <= 2 * n_alt, (c["pairs"], prod, n_alt)
    if n_alt == 0:
        assert c["pairs"] == prod


def product_form_counts(rec, W, H):
    """Total over pixels of the number of Gaussians in the included prefix
    (largest k with prod_{j<=k} (1 - a_j) >= T_min over the (z, index)-ordered
    candidates with a >= 1/255), alpha in FP64 from the projection records."""
    n = len(rec["u"])
    total = 0
    front = [g for g in range(n) if rec["in_front"][g]]
    order = sorted(front, key=lambda g: (rec["z"][g], g))
    for j in range(H):
        for i in range(W):
            prod = 1.0
            for g in order:
                dx = i + 0.5 - rec["u"][g]
                dy = j + 0.5 - rec["v"][g]
                q = rec["conic_a"][g] * dx * dx + 2 * rec["conic_b"][g] * dx * dy + \
                    rec["conic_c"][g] * dy * dy
                a = min(AMAX, rec["opacity"][g] * math.exp(-q / 2))
                if a < AMIN:
                    continue
                if prod * (1 - a) < TMIN:
                    break
                prod *= 1 - a
                total += 1
    return total
