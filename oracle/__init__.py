"""FP64 CPU oracle for the splat renderer -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, the smoke check and the benchmark's CPU-baseline leg may import
this package. It shares no code with the GPU renderer; both consume the seeded
arrays of `scenegen`.

`render()` wraps the C library built from `gs_oracle.c` (FP64 plain
definition of 3D Gaussian splat rendering with depth as a by-product,
Sec. 3.2 and Fig. "Rendering RGB and Depth"; splat model of the cited 3DGS,
Sec. 2.3). `compare()` is the comparator that accepts a GPU image when every
pixel matches the FP64 result, or one of the alternatives the oracle lists
for pixels whose decisions sit at a threshold within rounding.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Default margins: relative band around 1/255 for the skip test, relative
# band around 1e-4 for the stop test, absolute depth gap (m) for near-ties,
# absolute band (m) around the near plane.
DEFAULT_MARGINS = (2e-3, 2e-3, 2e-5, 1e-5)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.gso_quat_to_rot.argtypes = [dp, dp]
        L.gso_sh_basis.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        L.gso_sh_basis.restype = ctypes.c_double
        L.gso_sh_color.argtypes = [ctypes.c_int, dp, dp, dp]
        L.gso_project_all.argtypes = [fp, fp, fp, fp, fp, ctypes.c_int64, ctypes.c_int, fp, fp,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        L.gso_render.argtypes = [fp, fp, fp, fp, fp, ctypes.c_int64, ctypes.c_int, fp, fp,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, dp, dp,
                                 dp, dp, i64p, ctypes.c_int64, i32p, dp, i64p, ctypes.c_int]
        L.gso_render.restype = ctypes.c_int
        L.gso_pixel_trace.argtypes = [fp, fp, fp, fp, fp, ctypes.c_int64, ctypes.c_int, fp, fp,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.gso_pixel_trace.restype = ctypes.c_int
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def quat_to_rot(q) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9)
    lib().gso_quat_to_rot(_ptr(q, ctypes.c_double), _ptr(R, ctypes.c_double))
    return R.reshape(3, 3)


def sh_basis(l: int, m: int, d) -> float:
    d = np.ascontiguousarray(d, np.float64)
    return lib().gso_sh_basis(l, m, _ptr(d, ctypes.c_double))


def sh_color(deg: int, d, coef) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64)
    c = np.ascontiguousarray(coef, np.float64).reshape(-1)
    out = np.zeros(3)
    lib().gso_sh_color(deg, _ptr(d, ctypes.c_double), _ptr(c, ctypes.c_double),
                       _ptr(out, ctypes.c_double))
    return out


PROJ_FIELDS = ("u", "v", "z", "cov_a", "cov_b", "cov_c", "conic_a", "conic_b", "conic_c",
               "opacity", "r", "g", "b", "x0", "x1", "y0", "y1", "in_front", "visible",
               "projected")


def project_all(scene: dict, pose, intr, width: int, height: int, near: float = 0.2) -> dict:
    """Per-Gaussian FP64 projection records (u, v, z, 2D covariance, conic,
    colour, exact pixel box, flags) for one camera."""
    m, s, q, o, sh = (_f32(scene[k]) for k in ("means", "scales", "quats", "opacity", "sh"))
    n = len(o)
    out = np.zeros((n, 20))
    pose = _f32(pose).reshape(12)
    intr = _f32(intr).reshape(4)
    fp = ctypes.c_float
    lib().gso_project_all(_ptr(m, fp), _ptr(s, fp), _ptr(q, fp), _ptr(o, fp), _ptr(sh, fp), n,
                          int(scene["sh_degree"]), _ptr(pose, fp), _ptr(intr, fp), width,
                          height, float(np.float32(near)), _ptr(out, ctypes.c_double))
    return {k: out[:, i] for i, k in enumerate(PROJ_FIELDS)}


@dataclass
class Render:
    rgb: np.ndarray        # [H, W, 3] float64
    depth: np.ndarray      # [H, W]
    alpha: np.ndarray      # [H, W]  accumulated weight
    tfinal: np.ndarray     # [H, W]  transmittance after the walk
    counters: dict
    var_pix: np.ndarray    # [V] flattened pixel index of each alternative
    var_vals: np.ndarray   # [V, 5] r, g, b, depth, alpha


COUNTER_NAMES = ("projected", "visible", "instances16", "pairs", "flagged", "unresolved",
                 "candidates", "variants")


def render(scene: dict, pose, intr, width: int, height: int, near: float = 0.2,
           bg=(0.0, 0.0, 0.0), margins=DEFAULT_MARGINS, threads: int = 0) -> Render:
    """Render one camera with the FP64 oracle (see gs_oracle.c)."""
    m, s, q, o, sh = (_f32(scene[k]) for k in ("means", "scales", "quats", "opacity", "sh"))
    n = len(o)
    pose = _f32(pose).reshape(12)
    intr = _f32(intr).reshape(4)
    H, W = int(height), int(width)
    rgb = np.zeros((H, W, 3))
    depth = np.zeros((H, W))
    alpha = np.zeros((H, W))
    tfin = np.zeros((H, W))
    cnt = np.zeros(8, np.int64)
    bgv = np.ascontiguousarray(bg, np.float64)
    mar = np.ascontiguousarray(margins, np.float64)
    cap = max(1024, H * W // 4)
    fp, dp = ctypes.c_float, ctypes.c_double
    while True:
        vp = np.zeros(cap, np.int32)
        vv = np.zeros((cap, 5))
        nv = np.zeros(1, np.int64)
        rc = lib().gso_render(_ptr(m, fp), _ptr(s, fp), _ptr(q, fp), _ptr(o, fp), _ptr(sh, fp),
                              n, int(scene["sh_degree"]), _ptr(pose, fp), _ptr(intr, fp), W, H,
                              float(np.float32(near)), _ptr(bgv, dp), _ptr(mar, dp),
                              _ptr(rgb, dp), _ptr(depth, dp), _ptr(alpha, dp), _ptr(tfin, dp),
                              _ptr(cnt, ctypes.c_int64), cap, _ptr(vp, ctypes.c_int32),
                              _ptr(vv, dp), _ptr(nv, ctypes.c_int64), int(threads))
        if rc != 0:
            raise ValueError("oracle render rejected its arguments (rc=%d)" % rc)
        if nv[0] <= cap:
            break
        cap = int(nv[0]) + 16
    k = int(nv[0])
    order = np.argsort(vp[:k], kind="stable")
    return Render(rgb, depth, alpha, tfin, dict(zip(COUNTER_NAMES, cnt.tolist())),
                  vp[:k][order], vv[:k][order])


def blur_subposes(pose, velocity, shutter: float, n_sub: int) -> np.ndarray:
    """Camera poses of the sub-frames of a motion-blurred frame (Sec. 3.3 and
    the appendix figure on motion blur: frames offset along the camera's
    velocity, blended into one image). Reading: sub-frame k is the camera at
    the middle of the k-th of n_sub equal parts of the exposure [t - shutter,
    t], centre C - v (shutter (k + 1/2) / n_sub), rotation unchanged. The
    sub-frame poses are renderer inputs, so they are formed in FP32 (one
    rounded product and one rounded difference per coordinate)."""
    pose = _f32(pose).reshape(3, 4)
    v = _f32(velocity).reshape(3)
    out = np.repeat(pose[None], n_sub, axis=0)
    sh = float(np.float32(shutter))
    for k in range(n_sub):
        dt = np.float32(sh * (k + 0.5) / n_sub)
        out[k, :, 3] = pose[:, 3] - v * dt
    return out


def render_motion_blur(scene: dict, pose, velocity, intr, width: int, height: int,
                       shutter: float, n_sub: int, near: float = 0.2, bg=(0.0, 0.0, 0.0),
                       threads: int = 0):
    """Motion-blurred frame: the n_sub sub-frames rendered by `render` and
    blended with equal weights. Reading of the blend: RGB and accumulated
    weight are the means over the sub-frames; depth stays an expected depth,
    sum_k alpha_k depth_k / sum_k alpha_k (0 where every sub-frame is
    empty). Returns (rgb, depth, alpha, [per-sub-frame Render])."""
    subs = [render(scene, p, intr, width, height, near=near, bg=bg, threads=threads)
            for p in blur_subposes(pose, velocity, shutter, n_sub)]
    rgb = sum(r.rgb for r in subs) / n_sub
    asum = sum(r.alpha for r in subs)
    zsum = sum(r.alpha * r.depth for r in subs)
    depth = np.where(asum > 0, zsum / np.where(asum > 0, asum, 1.0), 0.0)
    return rgb, depth, asum / n_sub, subs


def pixel_trace(scene: dict, pose, intr, width: int, height: int, i: int, j: int,
                near: float = 0.2, eps_alpha: float = DEFAULT_MARGINS[0], cap: int = 256):
    """Candidates of pixel (i, j) in walk order: rows (g, z, alpha, T before,
    T after, flags). Diagnostic helper."""
    m, s, q, o, sh = (_f32(scene[k]) for k in ("means", "scales", "quats", "opacity", "sh"))
    out = np.zeros((cap, 6))
    pose = _f32(pose).reshape(12)
    intr = _f32(intr).reshape(4)
    fp = ctypes.c_float
    k = lib().gso_pixel_trace(_ptr(m, fp), _ptr(s, fp), _ptr(q, fp), _ptr(o, fp), _ptr(sh, fp),
                              len(o), int(scene["sh_degree"]), _ptr(pose, fp), _ptr(intr, fp),
                              width, height, float(np.float32(near)), eps_alpha, i, j, cap,
                              _ptr(out, ctypes.c_double))
    return out[:min(k, cap)]


# ------------------------------------------------------------- comparator ----

RGB_TOL = 2e-3      # max-abs RGB
DEPTH_TOL = 1e-3    # relative depth where the oracle's accumulated weight > 0
ALPHA_TOL = 2e-3    # max-abs accumulated weight


def _pixel_errors(ref_rgb, ref_depth, ref_alpha, rgb, depth, alpha):
    """Per-pixel errors; alpha None means the image has no alpha channel, so
    only RGB and depth are held to their tolerances."""
    e_rgb = np.max(np.abs(rgb - ref_rgb), axis=-1)
    has = ref_alpha > 0
    e_dep = np.where(has, np.abs(depth - ref_depth) / np.where(has, np.abs(ref_depth), 1.0),
                     np.abs(depth))
    e_alp = np.zeros_like(e_dep) if alpha is None else np.abs(alpha - ref_alpha)
    ok = (e_rgb <= RGB_TOL) & (e_dep <= DEPTH_TOL) & (e_alp <= ALPHA_TOL)
    return ok, e_rgb, e_dep, e_alp


def compare(ref: Render, rgb, depth, alpha=None) -> dict:
    """Compare one rendered camera against the oracle.

    A pixel passes when it is within tolerance of the FP64 result (max-abs
    RGB 2e-3, relative depth 1e-3, max-abs alpha 2e-3), or of one of the
    alternatives the oracle lists for that pixel. Without `alpha` only RGB
    and depth are compared (an alternative differs from the FP64 result in
    its accumulated weight too). Returns a report with the
    raw maxima, the maxima over the pixels that have no alternative
    (plain_*: only rounding separates the results there), the number of
    pixels with alternatives, flagged and unresolved by the oracle, accepted
    through an alternative (rescued) and failed."""
    rgb = np.asarray(rgb, np.float64)
    depth = np.asarray(depth, np.float64)
    alpha = None if alpha is None else np.asarray(alpha, np.float64)
    ok, e_rgb, e_dep, e_alp = _pixel_errors(ref.rgb, ref.depth, ref.alpha, rgb, depth, alpha)
    H, W = ref.depth.shape
    flat_ok = ok.reshape(-1)
    bad = np.nonzero(~flat_ok)[0]
    rescued = 0
    if len(bad) and len(ref.var_pix):
        starts = np.searchsorted(ref.var_pix, bad, side="left")
        ends = np.searchsorted(ref.var_pix, bad, side="right")
        rgb_f = rgb.reshape(-1, 3)
        dep_f = depth.reshape(-1)
        alp_f = None if alpha is None else alpha.reshape(-1)
        for p, a, b in zip(bad, starts, ends):
            if a == b:
                continue
            vv = ref.var_vals[a:b]
            okv, _, _, _ = _pixel_errors(vv[:, :3], vv[:, 3], vv[:, 4],
                                         rgb_f[p][None, :], dep_f[p],
                                         None if alp_f is None else alp_f[p])
            if okv.any():
                flat_ok[p] = True
                rescued += 1
    failed = int((~flat_ok).sum())
    # pixels for which the oracle lists no alternative: every decision there
    # is clear of its threshold, so only rounding separates the two results
    plain = np.ones(H * W, bool)
    plain[np.unique(ref.var_pix)] = False
    plain = plain.reshape(H, W)

    def pmax(e):
        return float(e[plain].max()) if plain.any() else 0.0
    return dict(max_abs_rgb=float(e_rgb.max()) if e_rgb.size else 0.0,
                max_rel_depth=float(e_dep.max()) if e_dep.size else 0.0,
                max_abs_alpha=float(e_alp.max()) if e_alp.size else 0.0,
                plain_max_abs_rgb=pmax(e_rgb), plain_max_rel_depth=pmax(e_dep),
                plain_max_abs_alpha=pmax(e_alp),
                with_alternatives=int(H * W - plain.sum()),
                flagged=int(ref.counters["flagged"]), unresolved=int(ref.counters["unresolved"]),
                rescued=rescued, failed=failed, pixels=H * W,
                failed_pixels=np.nonzero(~flat_ok)[0][:20].tolist())
