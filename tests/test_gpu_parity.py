"""GPU parity of the HIP renderer against the FP64 oracle, through the C ABI.

Tolerance (the renderer's stated bar): max-abs RGB 2e-3, relative depth
1e-3, max-abs alpha 2e-3 per pixel, after the comparator accepts pixels that
match an alternative the oracle lists for decisions sitting at a threshold
within rounding (oracle.compare).
"""
import math

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu


# Pixels for which the oracle lists no alternative have every decision clear
# of its threshold: there only FP32 rounding separates the GPU from the FP64
# result, and it is held to this much tighter bar.
PLAIN_TOL = 1e-4


def _check(ref, rgb, depth, alpha, label=""):
    rep = oracle.compare(ref, rgb, depth, alpha)
    print(f"{label}: max|rgb| {rep['max_abs_rgb']:.2e} rel depth {rep['max_rel_depth']:.2e} "
          f"|alpha| {rep['max_abs_alpha']:.2e}; plain pixels: |rgb| "
          f"{rep['plain_max_abs_rgb']:.2e} rel depth {rep['plain_max_rel_depth']:.2e} |alpha| "
          f"{rep['plain_max_abs_alpha']:.2e}; with alternatives {rep['with_alternatives']} "
          f"rescued {rep['rescued']} unresolved {rep['unresolved']} failed {rep['failed']}",
          flush=True)
    assert rep["failed"] == 0, (label, rep)
    assert rep["unresolved"] == 0, (label, rep)
    assert rep["rescued"] <= rep["with_alternatives"], (label, rep)
    assert rep["plain_max_abs_rgb"] <= PLAIN_TOL, (label, rep)
    assert rep["plain_max_rel_depth"] <= PLAIN_TOL, (label, rep)
    assert rep["plain_max_abs_alpha"] <= PLAIN_TOL, (label, rep)
    return rep


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def w0(gpu_renderer):
    sc = scenegen.make_scene(0)
    return sc, gpu_renderer.upload_scene(sc), scenegen.make_cameras(0)


@pytest.fixture(scope="module")
def w1(gpu_renderer):
    sc = scenegen.make_scene(1)
    return sc, gpu_renderer.upload_scene(sc), scenegen.make_cameras(1)


# ------------------------------------------------------------- projection --

@pytest.mark.parametrize("which", [0, 1])
def test_projection_records_match_oracle(gpu_renderer, w0, w1, which):
    sc, sid, cams = (w0, w1)[which]
    W, H = cams["width"], cams["height"]
    pose, intr = cams["poses"][0], cams["intrinsics"][0]
    got = gpu_renderer.debug_project(sid, pose, intr, W, H)
    ref = oracle.project_all(sc, pose, intr, W, H)
    vis_ref = ref["visible"] > 0
    vis_got = got[:, 14] > 0
    # the GPU's pixel box is widened by rounding margins: it may keep a few extra
    # Gaussians, never drop one the oracle sees
    assert np.all(vis_got[vis_ref]), np.nonzero(vis_ref & ~vis_got)[0][:10]
    assert (vis_got & ~vis_ref).sum() <= max(3, vis_ref.sum() // 1000)
    v = vis_ref
    np.testing.assert_allclose(got[v, 0], ref["u"][v], rtol=2e-6, atol=2e-3)
    np.testing.assert_allclose(got[v, 1], ref["v"][v], rtol=2e-6, atol=2e-3)
    np.testing.assert_allclose(got[v, 2], ref["z"][v], rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(got[v, 3], ref["opacity"][v], rtol=0, atol=0)
    for k, name in ((4, "conic_a"), (5, "conic_b"), (6, "conic_c")):
        scale = np.maximum(np.abs(ref["conic_a"][v]), np.abs(ref["conic_c"][v]))
        err = np.abs(got[v, k] - ref[name][v]) / scale
        assert err.max() < 1e-4, (name, err.max())
    for k, name in ((7, "r"), (8, "g"), (9, "b")):
        np.testing.assert_allclose(got[v, k], ref[name][v], atol=2e-5)
    # the GPU's pixel box contains the oracle's exact box
    assert np.all(got[v, 10] <= ref["x0"][v]) and np.all(got[v, 11] >= ref["x1"][v])
    assert np.all(got[v, 12] <= ref["y0"][v]) and np.all(got[v, 13] >= ref["y1"][v])
    # What the FP32 projection's errors do to alpha where the skip decision
    # is taken: on the oracle's alpha = 1/255 contour d^T Q d = r^2,
    # r^2 = 2 ln(255 o), the GPU's q differs by at most r^2 lambda_max (the
    # largest |eigenvalue| of Q^-1/2 dQ Q^-1/2) + 2 r |dmu|_Q, and alpha by
    # half that, relatively. The oracle's skip band (2e-3 of 1/255) must
    # hold it with room to spare: any pixel the two sides may decide
    # differently is then flagged.
    o = ref["opacity"][v]
    keep = o * 255.0 > 1.0 + 1e-3
    Qr = np.stack([ref["conic_a"][v], ref["conic_b"][v], ref["conic_b"][v], ref["conic_c"][v]],
                  -1).reshape(-1, 2, 2)[keep]
    dQ = (np.stack([got[v, 4], got[v, 5], got[v, 5], got[v, 6]], -1).reshape(-1, 2, 2)[keep]
          - Qr)
    dmu = np.stack([got[v, 0] - ref["u"][v], got[v, 1] - ref["v"][v]], -1)[keep]
    w, U = np.linalg.eigh(Qr)
    Qih = U @ (np.einsum("ni,nij->nij", 1.0 / np.sqrt(w), np.transpose(U, (0, 2, 1))))
    lam = np.abs(np.linalg.eigvalsh(Qih @ dQ @ Qih)).max(axis=1)
    r2 = 2.0 * np.log(255.0 * o[keep])
    mq = np.sqrt(np.einsum("ni,nij,nj->n", dmu, Qr, dmu))
    rel_alpha = 0.5 * (r2 * lam + 2.0 * np.sqrt(r2) * mq)
    print(f"workload {which}: alpha error on the 1/255 contour from the projection: max "
          f"{rel_alpha.max():.2e}, 99.9th percentile {np.percentile(rel_alpha, 99.9):.2e} "
          f"(skip band {oracle.DEFAULT_MARGINS[0]:.0e})", flush=True)
    assert rel_alpha.max() < oracle.DEFAULT_MARGINS[0] / 2


# -------------------------------------------------------------- workload 0 --

@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_workload0_matches_oracle(gpu_renderer, w0, mode):
    sc, sid, cams = w0
    rgb, depth, alpha = gpu_renderer.render([sid], cams["poses"], cams["intrinsics"], 64, 48,
                                            mode=mode)
    ref = oracle.render(sc, cams["poses"][0], cams["intrinsics"][0], 64, 48)
    _check(ref, _np(rgb[0]), _np(depth[0]), _np(alpha[0]), f"w0 {mode}")
    st = gpu_renderer.stats()
    assert st["visible"] == pytest.approx(ref.counters["visible"], rel=0.01)


# -------------------------------------------------------------- workload 1 --

def test_workload1_all_cameras_batched(gpu_renderer, w1):
    sc, sid, cams = w1
    n = len(cams["scene_ids"])
    rgb, depth, alpha = gpu_renderer.render([sid] * n, cams["poses"], cams["intrinsics"], 640, 480)
    rgb, depth, alpha = _np(rgb), _np(depth), _np(alpha)
    total_flag = 0
    for c in range(n):
        ref = oracle.render(sc, cams["poses"][c], cams["intrinsics"][c], 640, 480)
        _check(ref, rgb[c], depth[c], alpha[c], f"w1 cam {c}")
        total_flag += ref.counters["flagged"]
    print("w1 flagged pixels", total_flag)


def test_workload1_plain_equals_batched_bitwise(gpu_renderer, w1):
    sc, sid, cams = w1
    idx = np.arange(0, 64, 8)
    P, K = cams["poses"][idx], cams["intrinsics"][idx]
    a = gpu_renderer.render([sid] * len(idx), P, K, 640, 480, mode="plain")
    b = gpu_renderer.render([sid] * len(idx), P, K, 640, 480, mode="batched")
    for x, y in zip(a, b):
        assert bool((x == y).all())


@pytest.mark.parametrize("tile,batch,persistent", [((16, 16), 64, 0), ((32, 8), 128, 1),
                                                   ((8, 8), 64, 0), ((16, 8), 128, 1),
                                                   ((32, 16), 64, 0), ((16, 16), 256, 1),
                                                   ((32, 8), 64, 1)])
def test_every_tile_choice_is_bitwise_identical(gpu_renderer, w1, tile, batch, persistent):
    sc, sid, cams = w1
    idx = np.arange(0, 64, 4)
    P, K = cams["poses"][idx], cams["intrinsics"][idx]
    base = gpu_renderer.render([sid] * len(idx), P, K, 640, 480)
    alt = gpu_renderer.render([sid] * len(idx), P, K, 640, 480, tile=tile, lds_batch=batch,
                              persistent=persistent, chunk_cams=5)
    st = gpu_renderer.stats()
    assert (st["tile_w"], st["tile_h"], st["lds_batch"], st["persistent"]) == (*tile, batch,
                                                                              persistent)
    for x, y in zip(base, alt):
        assert bool((x == y).all())


def test_graph_replay_matches_eager_every_replay(gpu_renderer, w1):
    import torch
    sc, sid, cams = w1
    n = 16
    P = torch.as_tensor(cams["poses"][:n]).cuda()
    K = torch.as_tensor(cams["intrinsics"][:n]).cuda()
    eager = [_np(t) for t in gpu_renderer.render([sid] * n, P, K, 640, 480)]
    out = gpu_renderer.alloc_outputs(n, 640, 480)
    for rep in range(3):
        gpu_renderer.render([sid] * n, P, K, 640, 480, out=out, use_graph=True)
        torch.cuda.synchronize()
        for x, y in zip(eager, out):
            assert np.array_equal(x, _np(y)), f"replay {rep}"
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        del junk
    assert gpu_renderer.stats()["graph_captures"] >= 1


def test_graph_replay_tracks_new_poses(gpu_renderer, w1):
    import torch
    sc, sid, cams = w1
    n = 8
    P = torch.as_tensor(cams["poses"][:n]).cuda()
    K = torch.as_tensor(cams["intrinsics"][:n]).cuda()
    out = gpu_renderer.alloc_outputs(n, 640, 480)
    gpu_renderer.render([sid] * n, P, K, 640, 480, out=out, use_graph=True)
    P.copy_(torch.as_tensor(cams["poses"][8:8 + n]).cuda())   # same buffer, new poses
    gpu_renderer.render([sid] * n, P, K, 640, 480, out=out, use_graph=True)
    ref = gpu_renderer.render([sid] * n, cams["poses"][8:8 + n], cams["intrinsics"][8:8 + n],
                              640, 480)
    for x, y in zip(ref, out):
        assert bool((x == y).all())


def test_repeated_runs_bitwise_identical(gpu_renderer, w1):
    sc, sid, cams = w1
    a = gpu_renderer.render([sid] * 4, cams["poses"][:4], cams["intrinsics"][:4], 640, 480)
    b = gpu_renderer.render([sid] * 4, cams["poses"][:4], cams["intrinsics"][:4], 640, 480)
    for x, y in zip(a, b):
        assert bool((x == y).all())


# ------------------------------------------------------------- edge cases --

def test_ragged_image_and_single_pixel(gpu_renderer, w0):
    sc, sid, cams = w0
    for (W, H) in ((50, 37), (17, 1), (1, 1), (33, 65)):
        intr = np.array([[40.0, 40.0, W / 2, H / 2]], np.float32)
        rgb, depth, alpha = gpu_renderer.render([sid], cams["poses"], intr, W, H)
        ref = oracle.render(sc, cams["poses"][0], intr[0], W, H)
        _check(ref, _np(rgb[0]), _np(depth[0]), _np(alpha[0]), f"ragged {W}x{H}")


def test_camera_looking_away_is_empty(gpu_renderer, w0):
    sc, sid, cams = w0
    pose = cams["poses"].copy()
    pose[0, :, 2] *= -1   # flip forward axis: looks away from the cloud
    pose[0, :, 0] *= -1
    rgb, depth, alpha = gpu_renderer.render([sid], pose, cams["intrinsics"], 64, 48,
                                            bg=(0.25, 0.5, 0.75))
    assert np.allclose(_np(rgb[0]), [0.25, 0.5, 0.75]) and np.all(_np(depth[0]) == 0)
    assert np.all(_np(alpha[0]) == 0)


def test_camera_inside_cloud_near_plane(gpu_renderer, w0):
    sc, sid, cams = w0
    pose = cams["poses"].copy()
    pose[0, :, 3] = (0.1, -0.2, 0.0)   # inside the [-2,2]^3 cube
    rgb, depth, alpha = gpu_renderer.render([sid], pose, cams["intrinsics"], 64, 48)
    ref = oracle.render(sc, pose[0], cams["intrinsics"][0], 64, 48)
    _check(ref, _np(rgb[0]), _np(depth[0]), _np(alpha[0]), "inside")


@pytest.mark.parametrize("deg", [1, 2, 3])
def test_sh_degrees_and_background(gpu_renderer, deg):
    sc = scenegen.tiny_scene(300, 7 + deg, sh_degree=deg, spread=1.0)
    sid = gpu_renderer.upload_scene(sc, device_copy=(deg == 2))
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)[None].astype(np.float32)
    intr = np.array([[60.0, 60.0, 40.0, 30.0]], np.float32)
    bg = (0.1, 0.2, 0.3)
    rgb, depth, alpha = gpu_renderer.render([sid], pose, intr, 80, 60, bg=bg)
    ref = oracle.render(sc, pose[0], intr[0], 80, 60, bg=bg)
    _check(ref, _np(rgb[0]), _np(depth[0]), _np(alpha[0]), f"deg {deg}")
    gpu_renderer.release_scene(sid)


def test_single_gaussian_scene(gpu_renderer):
    sc = scenegen.tiny_scene(1, 3, sh_degree=0)
    sc["means"][:] = (0.0, 0.0, 3.0)
    sid = gpu_renderer.upload_scene(sc)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)[None].astype(np.float32)
    intr = np.array([[50.0, 50.0, 32.0, 24.0]], np.float32)
    rgb, depth, alpha = gpu_renderer.render([sid], pose, intr, 64, 48)
    ref = oracle.render(sc, pose[0], intr[0], 64, 48)
    _check(ref, _np(rgb[0]), _np(depth[0]), _np(alpha[0]), "n=1")
    gpu_renderer.release_scene(sid)


def test_many_scenes_mixed_batch(gpu_renderer):
    scenes = [scenegen.tiny_scene(200 + 150 * i, 40 + i, sh_degree=i % 4, spread=0.8)
              for i in range(5)]
    sids = [gpu_renderer.upload_scene(s) for s in scenes]
    rng = np.random.default_rng(0)
    n = 23
    pick = rng.integers(0, 5, size=n)
    poses = np.zeros((n, 3, 4), np.float32)
    poses[:, :, :3] = np.eye(3)
    poses[:, :, 3] = rng.uniform(-0.2, 0.2, size=(n, 3))
    intr = np.tile(np.array([[45.0, 45.0, 24.0, 20.0]], np.float32), (n, 1))
    out = gpu_renderer.render([sids[p] for p in pick], poses, intr, 48, 40, chunk_cams=4)
    for c in range(n):
        ref = oracle.render(scenes[pick[c]], poses[c], intr[c], 48, 40)
        _check(ref, _np(out[0][c]), _np(out[1][c]), _np(out[2][c]), f"mixed {c}")
    for s in sids:
        gpu_renderer.release_scene(s)


def test_capacity_regrow_path(gpu_renderer, w1):
    sc, sid, cams = w1
    ref = gpu_renderer.render([sid] * 4, cams["poses"][:4], cams["intrinsics"][:4], 640, 480)
    gpu_renderer.set_instance_capacity(1000)
    got = gpu_renderer.render([sid] * 4, cams["poses"][:4], cams["intrinsics"][:4], 640, 480)
    st = gpu_renderer.stats()
    assert st["regrows"] >= 1 and st["instance_capacity"] > 1000
    for x, y in zip(ref, got):
        assert bool((x == y).all())


def test_async_renders_back_to_back_equal_waiting_renders(gpu_renderer, w1):
    """Two renders of the same cameras with different poses enqueued back to
    back without waiting (eager and graph-replayed), one synchronisation,
    both outputs bitwise equal to renders that waited."""
    import torch
    sc, sid, cams = w1
    ids = [sid] * 8
    K = cams["intrinsics"][:8]
    Pa, Pb = cams["poses"][:8], cams["poses"][8:16]
    refs = [[t.cpu().numpy() for t in gpu_renderer.render(ids, P, K, 640, 480, sync=True)]
            for P in (Pa, Pb)]
    for use_graph in (False, True):
        P = torch.as_tensor(Pa).cuda()
        outs = [gpu_renderer.alloc_outputs(8, 640, 480) for _ in range(2)]
        gpu_renderer.render(ids, P, K, 640, 480, out=outs[0], use_graph=use_graph)  # sizes
        gpu_renderer.render(ids, P, K, 640, 480, out=outs[1], use_graph=use_graph)  # sizes
        P2 = torch.as_tensor(Pb).cuda()
        gpu_renderer.render(ids, P, K, 640, 480, out=outs[0], use_graph=use_graph)
        gpu_renderer.render(ids, P2, K, 640, 480, out=outs[1], use_graph=use_graph)
        torch.cuda.synchronize()
        gpu_renderer.status(wait=True)
        for ref, got in zip(refs, outs):
            for x, y in zip(ref, got):
                assert np.array_equal(x, y.cpu().numpy())
    gpu_renderer.drop_graphs()
    # the second render on another stream: it shares the context's work
    # buffers, so it must start only after the first (nothing else orders
    # them: the other stream waits only for the inputs, made before both)
    s2 = torch.cuda.Stream()
    for use_graph in (False, True):
        P, P2 = torch.as_tensor(Pa).cuda(), torch.as_tensor(Pb).cuda()
        outs = [gpu_renderer.alloc_outputs(8, 640, 480) for _ in range(2)]
        gpu_renderer.render(ids, P, K, 640, 480, out=outs[1], use_graph=use_graph)  # sizes
        torch.cuda.synchronize()
        s2.wait_stream(torch.cuda.current_stream())
        gpu_renderer.render(ids, P, K, 640, 480, out=outs[0], use_graph=use_graph)
        with torch.cuda.stream(s2):
            gpu_renderer.render(ids, P2, K, 640, 480, out=outs[1], use_graph=use_graph)
        torch.cuda.synchronize()
        gpu_renderer.status(wait=True)
        for ref, got in zip(refs, outs):
            for x, y in zip(ref, got):
                assert np.array_equal(x, y.cpu().numpy()), use_graph
    gpu_renderer.drop_graphs()


def test_async_overflow_is_reported_and_next_render_complete(gpu_renderer, w1):
    """A render that returns without waiting and overflows the instance
    buffers is reported by gs_render_status (GS_ERR_CAPACITY), which leaves
    the buffers grown: the next render is complete."""
    import paper_2510_15352_amd as gs
    sc, sid, cams = w1
    ids = [sid] * 4
    P, K = cams["poses"][:4], cams["intrinsics"][:4]
    # 100 m above the terrain looking up (+z): nothing in front of the cameras
    away = np.zeros_like(P)
    away[:, :, :3] = np.eye(3)
    away[:, 2, 3] = 100.0
    ref = [t.cpu().numpy() for t in gpu_renderer.render(ids, P, K, 640, 480, sync=True)]
    gpu_renderer.set_instance_capacity(1000)
    gpu_renderer.render(ids, away, K, 640, 480)        # first of the configuration: waits
    assert gpu_renderer.stats()["instances"] < 1000
    gpu_renderer.render(ids, P, K, 640, 480)           # does not wait; overflows
    with pytest.raises(gs.GsError) as e:
        gpu_renderer.status(wait=True)
    assert e.value.code == -4
    assert gpu_renderer.stats()["instance_capacity"] > 1000
    got = gpu_renderer.render(ids, P, K, 640, 480)
    gpu_renderer.status(wait=True)
    for x, y in zip(ref, got):
        assert np.array_equal(x, y.cpu().numpy())


def test_empty_cameras_between_visible_ones(gpu_renderer, w0):
    """Cameras with no visible Gaussian leave empty per-camera segments in the
    depth and tile sorts, here at the start, middle and end of chunks."""
    sc, sid, cams = w0
    away = cams["poses"][0].copy()
    away[:, 2] *= -1
    away[:, 0] *= -1
    poses = np.stack([away, cams["poses"][0], away, away, cams["poses"][0], away])
    intr = np.repeat(cams["intrinsics"][:1], len(poses), axis=0)
    ref = oracle.render(sc, cams["poses"][0], cams["intrinsics"][0], 64, 48)
    for chunk in (0, 2, 4):
        rgb, depth, alpha = gpu_renderer.render([sid] * len(poses), poses, intr, 64, 48,
                                                chunk_cams=chunk)
        for c in (1, 4):
            _check(ref, _np(rgb[c]), _np(depth[c]), _np(alpha[c]), f"chunk {chunk} cam {c}")
        for c in (0, 2, 3, 5):
            assert np.all(_np(alpha[c]) == 0) and np.all(_np(depth[c]) == 0)


def test_many_tiles_radix_path_matches_oracle(gpu_renderer, w0):
    """A camera with 21060 tiles (8x8 tiles on a 1296x1040 image): 15-bit
    tile keys, so the tile sort runs two 8-bit radix passes instead of the
    6 + 5 bits of a 640x480 image; checked against the oracle and, bitwise,
    against the 16x16 tiling."""
    sc, sid, cams = w0
    W, H = 1296, 1040
    intr = np.array([[900.0, 900.0, W / 2, H / 2]] * 2, np.float32)
    poses = np.repeat(cams["poses"][:1], 2, axis=0)
    poses[1, :, 3] += (0.3, -0.2, 0.5)
    small = gpu_renderer.render([sid] * 2, poses, intr, W, H, tile=(8, 8), lds_batch=64)
    big = gpu_renderer.render([sid] * 2, poses, intr, W, H, tile=(16, 16), lds_batch=128)
    for x, y in zip(small, big):
        assert bool((x == y).all())
    ref = oracle.render(sc, poses[1], intr[1], W, H)
    _check(ref, _np(small[0][1]), _np(small[1][1]), _np(small[2][1]), "8x8 1296x1040")


def test_camera_rate_decimation_renders_due_cameras_only(gpu_renderer, w1):
    """Over one period every camera is rendered exactly once, bitwise equal
    to the full render; slots of cameras not due keep their contents."""
    import torch
    sc, sid, cams = w1
    n, period = 13, 5
    P, K = cams["poses"][:n], cams["intrinsics"][:n]
    ids = [sid] * n
    full = gpu_renderer.render(ids, P, K, 640, 480)
    out = tuple(torch.full_like(t, -7.0) for t in full)
    seen = np.zeros(n, int)
    for step in range(period):
        before = [t.clone() for t in out]
        nd = gpu_renderer.render_due(ids, P, K, 640, 480, step, period, out, use_graph=(step % 2 == 0))
        due = [(step + i) % period == 0 for i in range(n)]
        assert nd == sum(due)
        for i in range(n):
            for t_new, t_old, t_full in zip(out, before, full):
                if due[i]:
                    assert bool((t_new[i] == t_full[i]).all())
                else:
                    assert bool((t_new[i] == t_old[i]).all())
        seen += due
    assert np.all(seen == 1)
    # explicit phases: all cameras due together at steps where step % 3 == 0
    out2 = tuple(torch.zeros_like(t) for t in full)
    assert gpu_renderer.render_due(ids, P, K, 640, 480, 4, 3, out2, phase=[2] * n) == n
    for a, b in zip(out2, full):
        assert bool((a == b).all())
    assert gpu_renderer.render_due(ids, P, K, 640, 480, 5, 3, out2, phase=[2] * n) == 0


def test_motion_blur_matches_oracle_sub_frames_and_blend(gpu_renderer, w1):
    """The blurred frame is the blend of its sub-frames: each sub-frame,
    rendered on its own at the oracle's FP32 sub-pose, matches the oracle,
    and the blurred output equals the blend of those sub-frames."""
    sc, sid, cams = w1
    n, K_sub, shutter = 2, 3, 0.04
    P, K = cams["poses"][:n], cams["intrinsics"][:n]
    vel = np.random.default_rng(5).normal(0.0, 2.0, size=(n, 3)).astype(np.float32)
    rgb, depth, alpha = gpu_renderer.render_motion_blur([sid] * n, P, vel, K, 640, 480,
                                                        shutter, K_sub)
    for c in range(n):
        sub = oracle.blur_subposes(P[c], vel[c], shutter, K_sub)
        g = gpu_renderer.render([sid] * K_sub, sub, np.repeat(K[c:c + 1], K_sub, axis=0), 640, 480)
        gr, gd, ga = _np(g[0]), _np(g[1]), _np(g[2])
        asum = ga.sum(0)
        np.testing.assert_allclose(_np(rgb[c]), gr.mean(0), atol=2e-6)
        np.testing.assert_allclose(_np(alpha[c]), asum / K_sub, atol=2e-6)
        want = np.where(asum > 0, (ga * gd).sum(0) / np.where(asum > 0, asum, 1), 0)
        np.testing.assert_allclose(_np(depth[c]), want, rtol=2e-5, atol=1e-6)
        for k in range(K_sub):
            ref = oracle.render(sc, sub[k], K[c], 640, 480)
            _check(ref, gr[k], gd[k], ga[k], f"blur cam {c} sub {k}")
        # and against the oracle's blend directly
        o_rgb, o_depth, o_alpha, _ = oracle.render_motion_blur(sc, P[c], vel[c], K[c], 640, 480,
                                                               shutter, K_sub)
        assert np.abs(_np(rgb[c]) - o_rgb).max() < oracle.RGB_TOL
        assert np.abs(_np(alpha[c]) - o_alpha).max() < oracle.ALPHA_TOL


def test_motion_blur_degenerate_cases(gpu_renderer, w1):
    """One sub-frame is the plain render at the mid-exposure pose, bitwise
    (and at the unmoved pose for a zero shutter); zero velocity gives the
    plain render up to the blend's rounding; graph replay equals eager."""
    sc, sid, cams = w1
    n = 3
    P, K = cams["poses"][:n], cams["intrinsics"][:n]
    vel = np.random.default_rng(6).normal(0.0, 2.0, size=(n, 3)).astype(np.float32)
    plain = gpu_renderer.render([sid] * n, P, K, 640, 480)
    mid = np.stack([oracle.blur_subposes(P[c], vel[c], 0.04, 1)[0] for c in range(n)])
    plain_mid = gpu_renderer.render([sid] * n, mid, K, 640, 480)
    one = gpu_renderer.render_motion_blur([sid] * n, P, vel, K, 640, 480, 0.04, 1)
    for x, y in zip(one, plain_mid):
        assert bool((x == y).all())
    zero = gpu_renderer.render_motion_blur([sid] * n, P, vel, K, 640, 480, 0.0, 1)
    for x, y in zip(zero, plain):
        assert bool((x == y).all())
    still = gpu_renderer.render_motion_blur([sid] * n, P, np.zeros((n, 3)), K, 640, 480, 0.04, 4,
                                            alpha=False)
    np.testing.assert_allclose(_np(still[0]), _np(plain[0]), atol=1e-6)
    np.testing.assert_allclose(_np(still[1]), _np(plain[1]), rtol=1e-5, atol=1e-6)
    eager = gpu_renderer.render_motion_blur([sid] * n, P, vel, K, 640, 480, 0.04, 4)
    for _ in range(3):
        graph = gpu_renderer.render_motion_blur([sid] * n, P, vel, K, 640, 480, 0.04, 4,
                                                use_graph=True)
        for x, y in zip(graph, eager):
            assert bool((x == y).all())


def test_peak_probes_are_plausible(gpu_renderer):
    """Measured FMA, exp and copy rates: positive and within the chip's
    published limits (39.3 T FP32 lane-ops/s without packing, 8 TB/s)."""
    fma, ex, cp = (gpu_renderer.peak_probe(k) for k in (0, 1, 2))
    print(f"FMA {fma / 1e12:.2f} T/s, exp {ex / 1e12:.2f} T/s, copy {cp / 1e12:.2f} TB/s")
    assert 5e12 < fma < 42e12
    assert 1e12 < ex <= fma * 1.05
    assert 1e12 < cp < 8.5e12


# ----------------------------------------------------------- error paths --

def test_error_codes(gpu_renderer, w0):
    import paper_2510_15352_amd as gs
    sc, sid, cams = w0
    with pytest.raises(gs.GsError) as e:
        gpu_renderer.render([sid + 100], cams["poses"], cams["intrinsics"], 64, 48)
    assert e.value.code == -1
    with pytest.raises(gs.GsError) as e:
        gpu_renderer.render([sid], cams["poses"], cams["intrinsics"], 0, 48)
    assert e.value.code == -1
    bad = dict(sc)
    bad["means"] = sc["means"].copy()
    bad["means"][5, 1] = np.nan
    with pytest.raises(gs.GsError) as e:
        gpu_renderer.upload_scene(bad)
    assert e.value.code == -2
    bad = dict(sc)
    bad["sh_degree"] = 4
    with pytest.raises(gs.GsError) as e:
        gpu_renderer.upload_scene(bad)
    assert e.value.code == -2
    with pytest.raises(gs.GsError) as e:
        gpu_renderer.render([sid], cams["poses"], cams["intrinsics"], 64, 48, tile=(24, 24))
    assert e.value.code == -1


def test_release_while_graph_holds_scene_is_busy(gpu_renderer):
    import paper_2510_15352_amd as gs
    sc = scenegen.tiny_scene(100, 99)
    sid = gpu_renderer.upload_scene(sc)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)[None].astype(np.float32)
    intr = np.array([[50.0, 50.0, 16.0, 16.0]], np.float32)
    gpu_renderer.render([sid], pose, intr, 32, 32, use_graph=True)
    with pytest.raises(gs.GsError) as e:
        gpu_renderer.release_scene(sid)
    assert e.value.code == -6
    gpu_renderer.drop_graphs()
    gpu_renderer.release_scene(sid)


@pytest.mark.parametrize("streams", [2, 4])
def test_multi_stream_pipelines_bitwise_equal_eager_and_graph(gpu_renderer, w1, streams):
    import torch
    sc, sid, cams = w1
    n = 20
    P = torch.as_tensor(cams["poses"][:n]).cuda()
    K = torch.as_tensor(cams["intrinsics"][:n]).cuda()
    one = [_np(t) for t in gpu_renderer.render([sid] * n, P, K, 640, 480, chunk_cams=3,
                                               streams=1)]
    many = [_np(t) for t in gpu_renderer.render([sid] * n, P, K, 640, 480, chunk_cams=3,
                                                streams=streams)]
    for x, y in zip(one, many):
        assert np.array_equal(x, y)
    out = gpu_renderer.alloc_outputs(n, 640, 480)
    for rep in range(3):
        gpu_renderer.render([sid] * n, P, K, 640, 480, out=out, chunk_cams=3, streams=streams,
                            use_graph=True)
        torch.cuda.synchronize()
        for x, y in zip(one, out):
            assert np.array_equal(x, _np(y)), f"replay {rep}"


def test_pair_and_visibility_counters_match_oracle(gpu_renderer, w0, w1):
    """The counters behind the roofline, against the oracle's (per camera):
    contributing (pixel, Gaussian) pairs equal up to the pixels with listed
    alternatives (each can differ by a few contributors); visible pairs and
    16x16-tile instances at least the oracle's exact-footprint counts (the
    GPU's pixel box is the exact box widened by a rounding margin) and at most a
    little above them."""
    for (sc, sid, cams), c, W, H in ((w0, 0, 64, 48), (w1, 5, 640, 480), (w1, 41, 640, 480)):
        gpu_renderer.render([sid], cams["poses"][c:c + 1], cams["intrinsics"][c:c + 1], W, H,
                            count_pairs=True, tile=(16, 16), lds_batch=128)
        st = gpu_renderer.stats()
        ref = oracle.render(sc, cams["poses"][c], cams["intrinsics"][c], W, H)
        n_alt = len(np.unique(ref.var_pix))
        rc = ref.counters
        print(f"{W}x{H} cam {c}: pairs GPU {st['pairs_contrib']} oracle {rc['pairs']} "
              f"(pixels with alternatives {n_alt}); visible {st['visible']} / {rc['visible']}; "
              f"instances {st['instances']} / {rc['instances16']}", flush=True)
        assert abs(st["pairs_contrib"] - rc["pairs"]) <= 3 * n_alt
        assert rc["visible"] <= st["visible"] <= rc["visible"] * 1.001 + 3
        assert rc["instances16"] <= st["instances"] <= rc["instances16"] * 1.01 + 3
        assert st["pairs_evaluated"] >= st["pairs_contrib"]
        assert st["pairs_issued"] >= st["pairs_evaluated"]
        # a pixel meets the same contributing records in the same order
        # whatever the batch size (the batches are culled against the live
        # pixels, so the evaluated pairs may differ)
        gpu_renderer.render([sid], cams["poses"][c:c + 1], cams["intrinsics"][c:c + 1], W, H,
                            count_pairs=True, tile=(16, 16), lds_batch=64)
        st64 = gpu_renderer.stats()
        assert st64["pairs_contrib"] == st["pairs_contrib"]
        assert st64["pairs_issued"] >= st64["pairs_evaluated"] >= st64["pairs_contrib"]


def test_trace_and_debug_modes(gpu_renderer, w0, capfd, monkeypatch):
    """GS_TRACE prints one line per render on stderr; GS_DEBUG waits after
    every stage of an eager render and checks for device errors. Neither
    changes a pixel."""
    import paper_2510_15352_amd as gs
    sc, sid, cams = w0
    ref = [_np(t) for t in gpu_renderer.render([sid], cams["poses"], cams["intrinsics"], 64, 48)]
    monkeypatch.setenv("GS_TRACE", "1")
    monkeypatch.setenv("GS_DEBUG", "1")
    r = gs.Renderer(0)
    try:
        s2 = r.upload_scene(sc)
        out = r.alloc_outputs(3, 64, 48)
        for use_graph in (False, True, True):
            got = r.render([s2] * 3, np.repeat(cams["poses"], 3, 0),
                           np.repeat(cams["intrinsics"], 3, 0), 64, 48, out=out,
                           use_graph=use_graph)
            for x, y in zip(ref, got):
                assert np.array_equal(x[0], _np(y[1]))
        err = capfd.readouterr().err
        lines = [l for l in err.splitlines() if l.startswith("[gs] render:")]
        print("\n".join(lines))
        assert len(lines) == 3
        assert "eager" in lines[0] and "graph captured" in lines[1] and "graph replayed" in lines[2]
    finally:
        r.close()


def test_extreme_gaussians_and_off_centre_principal_point(gpu_renderer):
    """Degenerate and extreme splats against the oracle: opacity exactly 1
    (alpha clamped to 0.99 at the centre), exactly fl32(1/255), just below it
    and 0; a Gaussian much larger than the view (the tangent clamp of the
    Jacobian); needles (one long axis, two of 1e-4 m) along the image
    diagonal and along the optical axis; sub-pixel Gaussians (1e-5 m: the
    0.3 px^2 low-pass sets their footprint); a Gaussian right at the near
    plane; with the principal point far off the image centre (asymmetric
    tangent clamp) and on it."""
    rng = np.random.default_rng(77)
    n_rand = 60
    sc = scenegen.tiny_scene(n_rand, 78, sh_degree=2, spread=0.7)
    special = []   # (mean, scales, quat, opacity)
    amin = float(np.float32(1.0 / 255.0))
    for o in (1.0, amin, float(np.nextafter(np.float32(amin), np.float32(0))), 0.0):
        special.append(((rng.uniform(-0.4, 0.4), rng.uniform(-0.3, 0.3), 2.5), (0.05, 0.03, 0.04),
                        (1.0, 0.0, 0.0, 0.0), o))
    special.append(((0.1, -0.1, 3.0), (12.0, 9.0, 10.0), (0.9, 0.1, 0.3, 0.2), 0.6))
    c, s_ = math.cos(math.pi / 8), math.sin(math.pi / 8)
    special.append(((0.0, 0.0, 2.8), (0.6, 1e-4, 1e-4), (c, 0.0, 0.0, s_), 0.9))   # diagonal
    special.append(((0.2, 0.1, 2.2), (1e-4, 1e-4, 0.8), (1.0, 0.0, 0.0, 0.0), 0.95))  # on axis
    for k in range(6):
        special.append(((rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4), rng.uniform(2, 4)),
                        (1e-5, 1e-5, 1e-5), (1.0, 0.0, 0.0, 0.0), 0.9))
    special.append(((0.05, 0.02, 0.2 + 2e-5), (0.05, 0.05, 0.05), (1.0, 0.0, 0.0, 0.0), 0.7))
    m = len(special)
    sc2 = dict(sh_degree=2)
    sc2["means"] = np.concatenate([sc["means"], np.array([s[0] for s in special])]).astype(np.float32)
    sc2["scales"] = np.concatenate([sc["scales"], np.array([s[1] for s in special])]).astype(np.float32)
    sc2["quats"] = np.concatenate([sc["quats"], np.array([s[2] for s in special])]).astype(np.float32)
    sc2["opacity"] = np.concatenate([sc["opacity"], np.array([s[3] for s in special])]).astype(np.float32)
    sc2["sh"] = np.concatenate([sc["sh"], rng.normal(0, 0.3, size=(m, 9, 3))]).astype(np.float32)
    assert float(sc2["opacity"][n_rand + 1]) == amin
    sid = gpu_renderer.upload_scene(sc2)
    try:
        pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
        poses = np.stack([pose, pose, pose])
        intr = np.array([[50.0, 50.0, 32.0, 24.0], [60.0, 45.0, 6.5, 41.0],
                         [40.0, 40.0, 58.0, 3.0]], np.float32)
        rgb, depth, alpha = gpu_renderer.render([sid] * 3, poses, intr, 64, 48)
        for k in range(3):
            ref = oracle.render(sc2, poses[k], intr[k], 64, 48)
            _check(ref, _np(rgb[k]), _np(depth[k]), _np(alpha[k]), f"extreme cam {k}")
    finally:
        gpu_renderer.release_scene(sid)


def test_live_pixel_culls_on_partly_saturated_blocks(gpu_renderer):
    """Stacks of three near-opaque splats in front saturate irregular patches
    of pixels, so many 8x8 blocks go on with only part of their pixels live
    while thousands of small splats behind still reach the rest. The walk
    culls against the live pixels (their rectangle; on tiles of at most two
    blocks also each record's box against the live lanes): every tile shape
    must give the same frames bit for bit on a ragged 72x56 image, and the
    oracle's. Every occluder sits at its own depth (no exact ties, which
    other tests cover)."""
    rng = np.random.default_rng(91)
    sc = scenegen.tiny_scene(3000, 92, sh_degree=0, spread=0.8, log_scale_mean=-3.2)
    occ = []
    for k in range(7):
        x, y = rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4)
        for dz in (0.0, 0.05, 0.1):
            occ.append(((x, y, 1.3 + 0.0137 * k + dz), (0.07, 0.05, 0.04), 0.97))
    m = len(occ)
    sc2 = dict(sh_degree=0)
    sc2["means"] = np.concatenate([sc["means"], np.array([o[0] for o in occ])]).astype(np.float32)
    sc2["scales"] = np.concatenate([sc["scales"], np.array([o[1] for o in occ])]).astype(np.float32)
    sc2["quats"] = np.concatenate([sc["quats"], np.tile([1.0, 0.0, 0.0, 0.0], (m, 1))]).astype(np.float32)
    sc2["opacity"] = np.concatenate([sc["opacity"], np.array([o[2] for o in occ])]).astype(np.float32)
    sc2["sh"] = np.concatenate([sc["sh"], rng.normal(0, 0.5, size=(m, 1, 3))]).astype(np.float32)
    sid = gpu_renderer.upload_scene(sc2)
    try:
        pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
        poses = np.stack([pose, pose])
        intr = np.array([[60.0, 60.0, 36.0, 28.0], [75.0, 70.0, 30.0, 25.0]], np.float32)
        W, H = 72, 56
        outs = {}
        for tile, batch in (((16, 16), 64), ((16, 8), 64), ((8, 8), 64), ((32, 8), 128)):
            outs[tile] = [_np(t) for t in gpu_renderer.render([sid] * 2, poses, intr, W, H,
                                                             tile=tile, lds_batch=batch,
                                                             persistent=0)]
        base = outs[(16, 16)]
        for tile, o in outs.items():
            for x, y in zip(base, o):
                assert np.array_equal(x, y), tile
        for k in range(2):
            stopped = float(np.mean(base[2][k] > 1.0 - 1e-3))
            print(f"partly saturated cam {k}: stopped pixels {stopped:.2f}", flush=True)
            assert 0.05 < stopped < 0.8
            ref = oracle.render(sc2, poses[k], intr[k], W, H)
            _check(ref, base[0][k], base[1][k], base[2][k], f"partly saturated cam {k}")
    finally:
        gpu_renderer.release_scene(sid)
