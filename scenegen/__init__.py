"""Seeded synthetic scenes and camera batches for the five renderer workloads.

This module only draws inputs: Gaussian parameters, per-camera scene indices,
camera-to-world poses and pinhole intrinsics. It holds none of the renderer's
arithmetic (projection, colour evaluation, compositing), so that the FP64
oracle and the GPU path can both consume its arrays without sharing code.

The paper renders real scans and video-model scenes (Sec. 3.1, Sec. 3.3); none
of those datasets exist here, so these generators stand in for them with the
sizes and value distributions of the five workloads:

  0  one 10k-Gaussian scene, SH degree 0, one 64x48 camera at (0,0,-5)
  1  one 200k-Gaussian terrain slab (20x20x3 m), SH degree 3,
     64 cameras at 640x480 on robot trajectories
  2  32 terrain scenes of log-uniform size in [50k, 1M], SH degree 3,
     4096 cameras at 640x480 (128 per scene, scene order shuffled)
  3  the workload-2 batch at 160x120 (intrinsics divided by 4)
  4  one 3M-Gaussian slab (50x50x5 m), SH degree 3, 8192 cameras at 320x240,
     100 consecutive trajectory steps

Conventions (shared with the C interface): poses are camera-to-world 3x4
row-major [R | C] with OpenCV camera axes (x right, y down, z forward);
quaternions are (w, x, y, z); scales are linear (exp of the drawn log-scales);
opacities are linear (sigmoid of the drawn logits); SH coefficients are
[n][(deg+1)^2][3], l-major with m = -l..l.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "WORKLOADS", "workload", "scene_sizes", "make_scene",
           "make_cameras", "camera_steps", "camera_trajectories", "tiny_scene"]


@dataclass(frozen=True)
class Workload:
    index: int
    name: str
    n_scenes: int
    sh_degree: int
    n_cams: int
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    extent: float = 0.0          # half-width of the terrain slab (m); 0 = cube
    zspan: float = 0.0           # heightfield range (m)
    n_fixed: int = 0             # Gaussians per scene when fixed
    n_range: tuple = (0, 0)      # log-uniform range of scene sizes
    steps: int = 1               # consecutive trajectory steps
    traj_steps: int = 500        # trajectory length cameras are sampled from
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    0: Workload(0, "cube10k_sh0_64x48", 1, 0, 1, 64, 48, 50.0, 50.0, 32.0, 24.0,
                n_fixed=10_000),
    1: Workload(1, "slab200k_sh3_64cams_640x480", 1, 3, 64, 640, 480,
                400.0, 400.0, 320.0, 240.0, extent=10.0, zspan=3.0,
                n_fixed=200_000),
    2: Workload(2, "32scenes_50k-1M_sh3_4096cams_640x480", 32, 3, 4096, 640, 480,
                400.0, 400.0, 320.0, 240.0, extent=10.0, zspan=3.0,
                n_range=(50_000, 1_000_000)),
    3: Workload(3, "32scenes_50k-1M_sh3_4096cams_160x120", 32, 3, 4096, 160, 120,
                100.0, 100.0, 80.0, 60.0, extent=10.0, zspan=3.0,
                n_range=(50_000, 1_000_000)),
    4: Workload(4, "slab3M_sh3_8192cams_320x240_100steps", 1, 3, 8192, 320, 240,
                200.0, 200.0, 160.0, 120.0, extent=25.0, zspan=5.0,
                n_fixed=3_000_000, steps=100),
}


def workload(k: int) -> Workload:
    return WORKLOADS[int(k)]


def _scene_seed(k: int, s: int) -> int:
    # workload 3 renders the workload-2 scenes, so it shares their seeds
    base = 2 if k == 3 else k
    return 1000 * base + s


def _camera_seed(k: int) -> int:
    base = 2 if k == 3 else k
    return 1000 * base + 999


def scene_sizes(k: int) -> list[int]:
    """Gaussian count of every scene of workload k."""
    w = workload(k)
    if w.n_fixed:
        return [w.n_fixed] * w.n_scenes
    rng = np.random.default_rng(_scene_seed(k, 997))
    lo, hi = w.n_range
    u = rng.uniform(math.log(lo), math.log(hi), size=w.n_scenes)
    return [int(round(math.exp(x))) for x in u]


# ---------------------------------------------------------------- terrain ----

@dataclass(frozen=True)
class Heightfield:
    amp: np.ndarray      # [8]
    freq: np.ndarray     # [8,2] cycles per metre
    phase: np.ndarray    # [8]
    lo: float
    hi: float
    zspan: float

    def __call__(self, x, y):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        h = np.zeros(np.broadcast(x, y).shape)
        for a, f, p in zip(self.amp, self.freq, self.phase):
            h += a * np.sin(2.0 * np.pi * (f[0] * x + f[1] * y) + p)
        return (h - self.lo) * (self.zspan / (self.hi - self.lo))


def heightfield(k: int, s: int) -> Heightfield:
    """Smooth random heightfield: 8 sinusoids, wavelengths 2-10 m, a_k ~ 1/k,
    rescaled so that its range over the slab is [0, zspan]."""
    w = workload(k)
    rng = np.random.default_rng(_scene_seed(k, s) + 500_000)
    lam = rng.uniform(2.0, 10.0, size=8)
    ang = rng.uniform(0.0, 2.0 * np.pi, size=8)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=8)
    amp = 1.0 / np.arange(1, 9, dtype=np.float64)
    freq = np.stack([np.cos(ang) / lam, np.sin(ang) / lam], axis=1)
    g = np.linspace(-w.extent, w.extent, 513)
    gx, gy = np.meshgrid(g, g)
    raw = np.zeros_like(gx)
    for a, f, p in zip(amp, freq, phase):
        raw += a * np.sin(2.0 * np.pi * (f[0] * gx + f[1] * gy) + p)
    return Heightfield(amp, freq, phase, float(raw.min()), float(raw.max()),
                       w.zspan)


# ----------------------------------------------------------------- scenes ----

def _attributes(rng, n, sh_degree, means):
    """Shared attribute draws (order: log-scales, quaternions, opacity
    logits, colour / SH); means are drawn by the caller first."""
    log_scales = rng.normal(-4.0, 0.5, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    ncoef = (sh_degree + 1) ** 2
    sh = np.zeros((n, ncoef, 3), np.float32)
    # DC coefficient chosen so that the degree-0 colour (coef * Y00 + 0.5)
    # equals the drawn rgb; Y00 = 1 / (2 sqrt(pi)).
    sh[:, 0, :] = (rgb - 0.5) * (2.0 * math.sqrt(math.pi))
    if ncoef > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.1, size=(n, ncoef - 1, 3))
    return dict(
        means=np.ascontiguousarray(means, np.float32),
        scales=np.exp(log_scales).astype(np.float32),
        quats=q.astype(np.float32),
        opacity=(1.0 / (1.0 + np.exp(-logits))).astype(np.float32),
        sh=sh,
        sh_degree=int(sh_degree),
    )


def make_scene(k: int, s: int = 0) -> dict:
    """Scene s of workload k as FP32 arrays (see module docstring)."""
    w = workload(k)
    n = scene_sizes(k)[s]
    rng = np.random.default_rng(_scene_seed(k, s))
    if w.extent == 0.0:
        means = rng.uniform(-2.0, 2.0, size=(n, 3))
    else:
        hf = heightfield(k, s)
        xy = rng.uniform(-w.extent, w.extent, size=(n, 2))
        means = np.concatenate([xy, hf(xy[:, 0], xy[:, 1])[:, None]], axis=1)
    return _attributes(rng, n, w.sh_degree, means)


def tiny_scene(n: int, seed: int, sh_degree: int = 0, spread: float = 0.6,
               log_scale_mean: float = -1.5) -> dict:
    """Small random scene in front of a camera at the origin looking along +z
    (means around z = 3), for brute-force and parity tests."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-spread, spread, n),
                      rng.uniform(-spread, spread, n),
                      rng.uniform(2.0, 4.0, n)], axis=1)
    sc = _attributes(rng, n, sh_degree, means)
    sc["scales"] = np.exp(rng.normal(log_scale_mean, 0.4, size=(n, 3))).astype(np.float32)
    return sc


# ---------------------------------------------------------------- cameras ----

def look_poses(positions, yaw, pitch_down):
    """Camera-to-world [R | C] (m x 3 x 4) for OpenCV axes (x right, y down,
    z forward); z-up world frame, roll 0."""
    positions = np.asarray(positions, np.float64).reshape(-1, 3)
    yaw = np.asarray(yaw, np.float64).reshape(-1)
    cp, sp = math.cos(pitch_down), math.sin(pitch_down)
    cy_, sy_ = np.cos(yaw), np.sin(yaw)
    fwd = np.stack([cy_ * cp, sy_ * cp, np.full_like(yaw, -sp)], axis=1)
    right = np.stack([sy_, -cy_, np.zeros_like(yaw)], axis=1)
    down = np.cross(fwd, right)
    return np.concatenate([np.stack([right, down, fwd], axis=2), positions[:, :, None]], axis=2)


def look_pose(position, yaw, pitch_down):
    """One camera-to-world pose (3x4), as look_poses."""
    return look_poses([position], [yaw], pitch_down)[0]


def _terrain_poses(k, scene_ids, pos, head):
    """Poses 0.5 m above each camera's scene heightfield, 15 degrees down."""
    z = np.empty(len(scene_ids))
    for s in np.unique(scene_ids):
        m = scene_ids == s
        z[m] = heightfield(k, int(s))(pos[m, 0], pos[m, 1]) + 0.5
    p3 = np.concatenate([pos, z[:, None]], axis=1)
    return look_poses(p3, head, math.radians(15.0))


def camera_trajectories(k: int, n_steps: int):
    """Positions (n_steps, n_cams, 2) and headings (n_steps, n_cams) of the
    seeded robot trajectories: 0.02 m forward per step, heading random walk
    N(0, 0.05^2), reflection at a 1 m margin of the slab."""
    w = workload(k)
    rng = np.random.default_rng(_camera_seed(k))
    lim = w.extent - 1.0
    pos = rng.uniform(-lim, lim, size=(w.n_cams, 2))
    head = rng.uniform(0.0, 2.0 * np.pi, size=w.n_cams)
    P = np.empty((n_steps, w.n_cams, 2))
    Hd = np.empty((n_steps, w.n_cams))
    for t in range(n_steps):
        P[t], Hd[t] = pos, head
        head = head + rng.normal(0.0, 0.05, size=w.n_cams)
        pos = pos + 0.02 * np.stack([np.cos(head), np.sin(head)], axis=1)
        for ax in (0, 1):
            hi = pos[:, ax] > lim
            lo = pos[:, ax] < -lim
            pos[hi, ax] = 2 * lim - pos[hi, ax]
            pos[lo, ax] = -2 * lim - pos[lo, ax]
            flip = hi | lo
            if ax == 0:
                head[flip] = np.pi - head[flip]
            else:
                head[flip] = -head[flip]
    return P, Hd


def make_cameras(k: int, step: int = 0, subset=None) -> dict:
    """Camera batch of workload k: scene_ids int32[n], poses f32[n,3,4],
    intrinsics f32[n,4] (fx, fy, cx, cy), width, height.

    Workloads 1-3 sample every camera at its own seeded trajectory step in
    [0, 500); workload 4 uses consecutive steps `step` = 0..99."""
    w = workload(k)
    n = w.n_cams
    rng = np.random.default_rng(_camera_seed(k) + 1)
    scene_ids = np.repeat(np.arange(w.n_scenes, dtype=np.int32), n // w.n_scenes)
    rng.shuffle(scene_ids)
    intr = np.tile(np.array([w.fx, w.fy, w.cx, w.cy], np.float32), (n, 1))
    poses = np.zeros((n, 3, 4), np.float64)
    if w.extent == 0.0:
        poses[:, :, :3] = np.eye(3)
        poses[:, :, 3] = (0.0, 0.0, -5.0)
    else:
        if w.steps > 1:
            P, Hd = camera_trajectories(k, step + 1)
            pos, head = P[step], Hd[step]
        else:
            P, Hd = camera_trajectories(k, w.traj_steps)
            pick = rng.integers(0, w.traj_steps, size=n)
            pos, head = P[pick, np.arange(n)], Hd[pick, np.arange(n)]
        poses = _terrain_poses(k, scene_ids, pos, head)
    out = dict(scene_ids=scene_ids, poses=poses.astype(np.float32),
               intrinsics=intr, width=w.width, height=w.height)
    if subset is not None:
        idx = np.asarray(subset)
        out["scene_ids"] = out["scene_ids"][idx]
        out["poses"] = out["poses"][idx]
        out["intrinsics"] = out["intrinsics"][idx]
    return out


def camera_steps(k: int, n_steps: int) -> dict:
    """Consecutive sim steps 0..n_steps-1 of workload k's trajectories:
    poses f32[n_steps, n, 3, 4]; step t equals make_cameras(k, t)."""
    w = workload(k)
    base = make_cameras(k, 0)
    P, Hd = camera_trajectories(k, n_steps)
    poses = np.empty((n_steps, w.n_cams, 3, 4), np.float32)
    for t in range(n_steps):
        poses[t] = _terrain_poses(k, base["scene_ids"], P[t], Hd[t]).astype(np.float32)
    return dict(scene_ids=base["scene_ids"], poses=poses, intrinsics=base["intrinsics"],
                width=w.width, height=w.height)


def sampled_cameras(k: int, count: int, seed: int) -> dict:
    """`count` independent cameras over the scenes of workload k (training
    and calibration sets of the learned upsampler): scene uniform, position
    uniform over the slab minus a 1 m margin, heading uniform, 0.5 m above
    the heightfield, 15 degrees down. Seeds are offset so they never
    coincide with the evaluation trajectories."""
    w = workload(k)
    rng = np.random.default_rng(7_000_000 + 1000 * seed + k)
    lim = w.extent - 1.0
    sids = rng.integers(0, w.n_scenes, size=count).astype(np.int32)
    pos = rng.uniform(-lim, lim, size=(count, 2))
    head = rng.uniform(0.0, 2.0 * np.pi, size=count)
    poses = _terrain_poses(k, sids, pos, head)
    intr = np.tile(np.array([w.fx, w.fy, w.cx, w.cy], np.float32), (count, 1))
    return dict(scene_ids=sids, poses=poses.astype(np.float32), intrinsics=intr,
                width=w.width, height=w.height)


def camera_subset(k: int, count: int, seed: int = 12345) -> np.ndarray:
    """Seeded subset of camera indices of workload k (sorted)."""
    rng = np.random.default_rng(seed + k)
    return np.sort(rng.choice(workload(k).n_cams, size=count, replace=False))
