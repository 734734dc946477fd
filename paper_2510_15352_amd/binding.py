"""ctypes binding of libgsmi.so (the C interface in include/gs.h).

Argument marshalling only: PyTorch provides device memory and the current
HIP stream; every step of rendering runs in the library's HIP kernels.
Importing works without a GPU (the library loads; nothing is launched), and
every entry point raises if the library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsmi.so")

GS_OK = 0
ERRORS = {-1: "GS_ERR_INVALID_ARG", -2: "GS_ERR_BAD_SCENE", -3: "GS_ERR_OOM",
          -4: "GS_ERR_CAPACITY", -5: "GS_ERR_HIP", -6: "GS_ERR_BUSY", -7: "GS_ERR_NOT_TRAINED"}
GS_MEM_HOST, GS_MEM_DEVICE = 0, 1
GS_MODE_PLAIN, GS_MODE_BATCHED = 0, 1

# every symbol include/gs.h declares
EXPORTS = ("gs_abi_sizes", "gs_default_opts", "gs_create", "gs_destroy", "gs_last_error", "gs_upload_scene",
           "gs_release_scene", "gs_scene_size", "gs_render_batch", "gs_render_due",
           "gs_render_batch_motion_blur", "gs_render_backward", "gs_peak_probe",
           "gs_last_stats", "gs_render_status",
           "gs_debug_project", "gs_autotune", "gs_set_instance_capacity", "gs_clear_graphs",
           "gs_upsampler_num_params", "gs_upsampler_init", "gs_upsampler_set_weights",
           "gs_upsampler_get_weights", "gs_upsampler_save", "gs_upsampler_load",
           "gs_upsampler_forward", "gs_upsampler_forward_noalloc", "gs_upsampler_grads", "gs_upsampler_step",
           "gs_upsampler_apply_grads", "gs_upsampler_get_state", "gs_upsampler_lr",
           "gs_upsampler_score", "gs_upsampler_train", "gs_render_batch_upsampled", "gs_frame_psnr")


class GsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class SceneDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("mem_kind", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("near_plane", ctypes.c_float), ("bg", ctypes.c_float * 3), ("mode", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("lds_batch", ctypes.c_int32), ("chunk_cams", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("count_pairs", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("sync", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 1)]

class TrainOpts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("steps", ctypes.c_int32), ("lr", ctypes.c_float),
                ("lr_min", ctypes.c_float), ("reserved", ctypes.c_int32 * 4)]


STAGES = ("setup", "project", "compact", "depth_sort", "emit", "tile_sort", "ranges", "raster")


class Stats(ctypes.Structure):
    _fields_ = [("visible", ctypes.c_int64), ("instances", ctypes.c_int64),
                ("instance_capacity", ctypes.c_int64), ("regrows", ctypes.c_int32),
                ("graph_captures", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("lds_batch", ctypes.c_int32),
                ("chunk_cams", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("stage_launches", ctypes.c_int32 * 8), ("stage_ms", ctypes.c_float * 8),
                ("pairs_contrib", ctypes.c_int64), ("pairs_evaluated", ctypes.c_int64),
                ("pairs_issued", ctypes.c_int64)]


_lib = None


def load():
    """Load libgsmi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python paper_2510_15352_amd/build.py` (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, fp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.gs_default_opts.argtypes = [ctypes.POINTER(RenderOpts)]
    L.gs_default_opts.restype = None
    L.gs_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    L.gs_destroy.argtypes = [vp]
    L.gs_last_error.argtypes = [vp]
    L.gs_last_error.restype = ctypes.c_char_p
    L.gs_upload_scene.argtypes = [vp, ctypes.POINTER(SceneDesc), ctypes.POINTER(i32)]
    L.gs_release_scene.argtypes = [vp, i32]
    L.gs_scene_size.argtypes = [vp, i32]
    L.gs_scene_size.restype = i64
    L.gs_render_batch.argtypes = [vp, i32, vp, vp, vp, i32, i32, vp, vp, vp,
                                  ctypes.POINTER(RenderOpts), vp]
    L.gs_render_due.argtypes = [vp, i32, vp, vp, vp, i32, i32, i64, i32, vp, vp, vp, vp,
                                ctypes.POINTER(RenderOpts), ctypes.POINTER(i32), vp]
    L.gs_render_batch_motion_blur.argtypes = [vp, i32, vp, vp, vp, vp, i32, i32, fp, i32, vp, vp,
                                              vp, ctypes.POINTER(RenderOpts), vp]
    L.gs_render_backward.argtypes = [vp, i32, i32, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp,
                                     vp, vp, vp]
    L.gs_peak_probe.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    L.gs_last_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.gs_render_status.argtypes = [vp, i32]
    L.gs_debug_project.argtypes = [vp, i32, vp, vp, i32, i32, fp, vp]
    L.gs_autotune.argtypes = [vp, i32, vp, vp, vp, i32, i32, vp, vp, ctypes.c_char_p, vp]
    L.gs_set_instance_capacity.argtypes = [vp, i64]
    L.gs_clear_graphs.argtypes = [vp]
    L.gs_upsampler_num_params.argtypes = []
    L.gs_upsampler_num_params.restype = i64
    L.gs_upsampler_init.argtypes = [vp, ctypes.c_uint64]
    L.gs_upsampler_set_weights.argtypes = [vp, vp, i64]
    L.gs_upsampler_get_weights.argtypes = [vp, vp, i64]
    L.gs_upsampler_save.argtypes = [vp, ctypes.c_char_p]
    L.gs_upsampler_load.argtypes = [vp, ctypes.c_char_p]
    L.gs_upsampler_forward.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
    L.gs_upsampler_forward_noalloc.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
    L.gs_upsampler_grads.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.gs_upsampler_step.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, fp, vp, vp]
    L.gs_upsampler_apply_grads.argtypes = [vp, vp, i64, fp]
    L.gs_upsampler_get_state.argtypes = [vp, vp, vp, i64, ctypes.POINTER(i32)]
    L.gs_upsampler_lr.argtypes = [i32, i32, fp, fp]
    L.gs_upsampler_lr.restype = fp
    L.gs_upsampler_score.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
    L.gs_upsampler_train.argtypes = [vp, ctypes.POINTER(TrainOpts), i32, vp, vp, vp, i32, i32, vp,
                                     vp]
    L.gs_render_batch_upsampled.argtypes = [vp, i32, vp, vp, vp, i32, i32, vp, vp, vp,
                                            ctypes.c_float, vp, ctypes.POINTER(RenderOpts), vp]
    L.gs_frame_psnr.argtypes = [vp, i32, i64, vp, vp, vp, vp]
    for name in EXPORTS:
        if not hasattr(L, name):
            raise RuntimeError(f"{LIB_PATH} does not export {name}")
    sizes = [ctypes.c_int32() for _ in range(3)]
    L.gs_abi_sizes(*[ctypes.byref(s) for s in sizes])
    mine = (ctypes.sizeof(SceneDesc), ctypes.sizeof(RenderOpts), ctypes.sizeof(Stats))
    if tuple(s.value for s in sizes) != mine:
        raise RuntimeError(f"struct layout mismatch: library {[s.value for s in sizes]}, "
                           f"binding {list(mine)}")
    _lib = L
    return L


def _stream_ptr(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f32(torch, a, device):
    t = torch.as_tensor(a)
    return t.to(device=device, dtype=torch.float32).contiguous()


class Renderer:
    """A gs_ctx on one HIP device."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the renderer runs only on the GPU")
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        rc = self.lib.gs_create(device, ctypes.byref(h))
        if rc != GS_OK:
            raise GsError(rc, "gs_create failed")
        self.ctx = h
        self._keep = {}

    # ------------------------------------------------------------ errors --
    def _check(self, rc):
        if rc < 0:
            raise GsError(rc, self.lib.gs_last_error(self.ctx).decode())
        return rc

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.gs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ scenes --
    def upload_scene(self, scene: dict, device_copy: bool = False) -> int:
        """Upload a scene (dict of FP32 arrays, see scenegen). With
        device_copy the arrays are first placed in device memory and the
        library reads them there (GS_MEM_DEVICE)."""
        torch = self.torch
        n = int(len(scene["opacity"]))
        keys = ("means", "scales", "quats", "opacity", "sh")
        if device_copy:
            arrs = [_dev_f32(torch, scene[k], self.device) for k in keys]
            ptrs = [a.data_ptr() for a in arrs]
            kind = GS_MEM_DEVICE
        else:
            arrs = [np.ascontiguousarray(np.asarray(scene[k]), dtype=np.float32) for k in keys]
            ptrs = [a.ctypes.data for a in arrs]
            kind = GS_MEM_HOST
        d = SceneDesc(n, int(scene["sh_degree"]), kind, *ptrs)
        sid = ctypes.c_int32(-1)
        self._check(self.lib.gs_upload_scene(self.ctx, ctypes.byref(d), ctypes.byref(sid)))
        self._keep[("deg", sid.value)] = int(scene["sh_degree"])
        return sid.value

    def release_scene(self, sid: int):
        self._check(self.lib.gs_release_scene(self.ctx, sid))

    def scene_size(self, sid: int) -> int:
        return self._check(self.lib.gs_scene_size(self.ctx, sid))

    # ------------------------------------------------------------ render --
    def opts(self, mode="batched", tile=None, lds_batch=0, chunk_cams=0, persistent=-1,
             use_graph=False, near=0.2, bg=(0.0, 0.0, 0.0), timing=False, count_pairs=False,
             streams=0, sync=False):
        o = RenderOpts()
        self.lib.gs_default_opts(ctypes.byref(o))
        o.mode = GS_MODE_PLAIN if mode == "plain" else GS_MODE_BATCHED
        if tile:
            o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
        o.lds_batch = int(lds_batch)
        o.chunk_cams = int(chunk_cams)
        o.persistent = int(persistent)
        o.use_graph = int(bool(use_graph))
        o.timing = int(bool(timing))
        o.count_pairs = int(bool(count_pairs))
        o.streams = int(streams)
        o.sync = int(bool(sync))
        o.near_plane = float(near)
        for i in range(3):
            o.bg[i] = float(bg[i])
        return o

    def alloc_outputs(self, n_cams, width, height, alpha=True):
        torch = self.torch
        rgb = torch.empty((n_cams, height, width, 3), dtype=torch.float32, device=self.device)
        depth = torch.empty((n_cams, height, width), dtype=torch.float32, device=self.device)
        al = (torch.empty((n_cams, height, width), dtype=torch.float32, device=self.device)
              if alpha else None)
        return rgb, depth, al

    def render(self, scene_ids, poses, intrinsics, width, height, out=None, alpha=True,
               opts=None, **kw):
        """Render; returns (rgb, depth, alpha) device tensors. `poses` and
        `intrinsics` may be numpy or torch (moved to the device)."""
        torch = self.torch
        sids = np.ascontiguousarray(np.asarray(scene_ids, dtype=np.int32).reshape(-1))
        n = len(sids)
        P = poses if (torch.is_tensor(poses) and poses.is_cuda and poses.dtype == torch.float32
                      and poses.is_contiguous()) else _dev_f32(torch, poses, self.device)
        K = intrinsics if (torch.is_tensor(intrinsics) and intrinsics.is_cuda
                           and intrinsics.dtype == torch.float32 and intrinsics.is_contiguous()) \
            else _dev_f32(torch, intrinsics, self.device)
        if P.numel() != n * 12 or K.numel() != n * 4:
            raise ValueError("poses must be [n,3,4] and intrinsics [n,4]")
        rgb, depth, al = out if out is not None else self.alloc_outputs(n, width, height, alpha)
        o = opts if opts is not None else self.opts(**kw)
        self._check(self.lib.gs_render_batch(
            self.ctx, n, sids.ctypes.data, P.data_ptr(), K.data_ptr(), int(width), int(height),
            rgb.data_ptr(), depth.data_ptr(), al.data_ptr() if al is not None else None,
            ctypes.byref(o), _stream_ptr(torch)))
        return rgb, depth, al

    def render_backward(self, scene_id, poses, intrinsics, width, height, grad_rgb=None,
                        grad_depth=None, grad_alpha=None, opts=None, **kw):
        """Gradients of sum(grad_rgb * rgb) + sum(grad_depth * depth) +
        sum(grad_alpha * alpha) over the cameras' renders of one scene with
        respect to its parameters; returns a dict of device tensors (means,
        scales, quats, opacity, sh) in the scene's upload order."""
        torch = self.torch
        P, K = self._dev(poses), self._dev(intrinsics)
        n = P.numel() // 12
        if P.numel() != n * 12 or K.numel() != n * 4 or n < 1:
            raise ValueError("poses must be [n,3,4] and intrinsics [n,4]")
        ups = []
        for t, last in ((grad_rgb, 3), (grad_depth, None), (grad_alpha, None)):
            if t is None:
                ups.append(None)
                continue
            t = self._dev(t)
            want = n * height * width * (last or 1)
            if t.numel() != want:
                raise ValueError("upstream gradients must be [n,H,W,3] / [n,H,W]")
            ups.append(t)
        N = self.scene_size(scene_id)
        nc = (self._keep[("deg", int(scene_id))] + 1) ** 2
        dev = self.device
        out = {"means": torch.empty((N, 3), dtype=torch.float32, device=dev),
               "scales": torch.empty((N, 3), dtype=torch.float32, device=dev),
               "quats": torch.empty((N, 4), dtype=torch.float32, device=dev),
               "opacity": torch.empty((N,), dtype=torch.float32, device=dev),
               "sh": torch.empty((N, nc, 3), dtype=torch.float32, device=dev)}
        o = opts if opts is not None else self.opts(**kw)
        self._check(self.lib.gs_render_backward(
            self.ctx, int(scene_id), n, P.data_ptr(), K.data_ptr(), int(width), int(height),
            *[u.data_ptr() if u is not None else None for u in ups], ctypes.byref(o),
            out["means"].data_ptr(), out["scales"].data_ptr(), out["quats"].data_ptr(),
            out["opacity"].data_ptr(), out["sh"].data_ptr(), _stream_ptr(torch)))
        return out

    def render_motion_blur(self, scene_ids, poses, velocities, intrinsics, width, height,
                           shutter, n_sub, out=None, alpha=True, opts=None, **kw):
        """Motion-blurred render: n_sub sub-frames along each camera's
        velocity over the shutter interval, blended; returns (rgb, depth,
        alpha) device tensors."""
        torch = self.torch
        sids = np.ascontiguousarray(np.asarray(scene_ids, dtype=np.int32).reshape(-1))
        n = len(sids)
        P = _dev_f32(torch, poses, self.device)
        V = _dev_f32(torch, velocities, self.device)
        K = _dev_f32(torch, intrinsics, self.device)
        if P.numel() != n * 12 or K.numel() != n * 4 or V.numel() != n * 3:
            raise ValueError("poses [n,3,4], velocities [n,3] and intrinsics [n,4] expected")
        rgb, depth, al = out if out is not None else self.alloc_outputs(n, width, height, alpha)
        o = opts if opts is not None else self.opts(**kw)
        self._check(self.lib.gs_render_batch_motion_blur(
            self.ctx, n, sids.ctypes.data, P.data_ptr(), V.data_ptr(), K.data_ptr(), int(width),
            int(height), float(shutter), int(n_sub), rgb.data_ptr(), depth.data_ptr(),
            al.data_ptr() if al is not None else None, ctypes.byref(o), _stream_ptr(torch)))
        return rgb, depth, al

    def render_due(self, scene_ids, poses, intrinsics, width, height, sim_step, period,
                   out, phase=None, opts=None, **kw):
        """Camera-rate decimation: render only the cameras due at `sim_step`
        into `out` (rgb, depth, alpha), leaving the other slots untouched;
        returns the number of cameras rendered."""
        torch = self.torch
        sids = np.ascontiguousarray(np.asarray(scene_ids, dtype=np.int32).reshape(-1))
        n = len(sids)
        P = poses if (torch.is_tensor(poses) and poses.is_cuda and poses.dtype == torch.float32
                      and poses.is_contiguous()) else _dev_f32(torch, poses, self.device)
        K = intrinsics if (torch.is_tensor(intrinsics) and intrinsics.is_cuda
                           and intrinsics.dtype == torch.float32 and intrinsics.is_contiguous()) \
            else _dev_f32(torch, intrinsics, self.device)
        if P.numel() != n * 12 or K.numel() != n * 4:
            raise ValueError("poses must be [n,3,4] and intrinsics [n,4]")
        ph = None
        if phase is not None:
            ph = np.ascontiguousarray(np.asarray(phase, dtype=np.int32).reshape(-1))
            if len(ph) != n:
                raise ValueError("phase must hold one value per camera")
        rgb, depth, al = out
        o = opts if opts is not None else self.opts(**kw)
        nd = ctypes.c_int32(0)
        self._check(self.lib.gs_render_due(
            self.ctx, n, sids.ctypes.data, P.data_ptr(), K.data_ptr(), int(width), int(height),
            int(sim_step), int(period), ph.ctypes.data if ph is not None else None,
            rgb.data_ptr(), depth.data_ptr(), al.data_ptr() if al is not None else None,
            ctypes.byref(o), ctypes.byref(nd), _stream_ptr(torch)))
        return nd.value

    def status(self, wait: bool = True):
        """gs_render_status: raises GsError (GS_ERR_CAPACITY) when a render
        that returned without waiting overflowed its instance buffers."""
        self._check(self.lib.gs_render_status(self.ctx, int(bool(wait))))

    def peak_probe(self, kind: int) -> float:
        """Measured rate: 0 FMA lane-ops/s, 1 v_exp_f32 lane-ops/s, 2 copy bytes/s."""
        v = ctypes.c_double(0.0)
        self._check(self.lib.gs_peak_probe(self.ctx, int(kind), ctypes.byref(v)))
        return v.value

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.gs_last_stats(self.ctx, ctypes.byref(s)))
        out = {k: getattr(s, k) for k, _ in Stats._fields_
               if k not in ("stage_ms", "stage_launches")}
        out["stage_ms"] = dict(zip(STAGES, list(s.stage_ms)))
        out["stage_launches"] = dict(zip(STAGES, list(s.stage_launches)))
        return out

    def set_instance_capacity(self, cap: int):
        self._check(self.lib.gs_set_instance_capacity(self.ctx, int(cap)))

    def drop_graphs(self):
        self._check(self.lib.gs_clear_graphs(self.ctx))

    def debug_project(self, sid, pose, intr, width, height, near=0.2):
        """Per-Gaussian projection records of one camera: [n, 16] numpy."""
        torch = self.torch
        n = self.scene_size(sid)
        out = torch.empty((n, 16), dtype=torch.float32, device=self.device)
        p = np.ascontiguousarray(np.asarray(pose, np.float32).reshape(12))
        k = np.ascontiguousarray(np.asarray(intr, np.float32).reshape(4))
        self._check(self.lib.gs_debug_project(self.ctx, sid, p.ctypes.data, k.ctypes.data,
                                              int(width), int(height), float(near),
                                              out.data_ptr()))
        return out.cpu().numpy()

    # --------------------------------------------------------- upsampler --
    def up_num_params(self) -> int:
        return int(self.lib.gs_upsampler_num_params())

    def up_init(self, seed: int = 0):
        self._check(self.lib.gs_upsampler_init(self.ctx, int(seed)))

    def up_set(self, params):
        p = np.ascontiguousarray(np.asarray(params, np.float32).reshape(-1))
        self._check(self.lib.gs_upsampler_set_weights(self.ctx, p.ctypes.data, len(p)))

    def up_get(self):
        p = np.zeros(self.up_num_params(), np.float32)
        self._check(self.lib.gs_upsampler_get_weights(self.ctx, p.ctypes.data, len(p)))
        return p

    def up_save(self, path):
        self._check(self.lib.gs_upsampler_save(self.ctx, os.fsencode(path)))

    def up_load(self, path):
        self._check(self.lib.gs_upsampler_load(self.ctx, os.fsencode(path)))

    def up_forward(self, rgb_lo, depth_lo):
        torch = self.torch
        n, h, w, _ = rgb_lo.shape
        rgb = torch.empty((n, 4 * h, 4 * w, 3), dtype=torch.float32, device=self.device)
        depth = torch.empty((n, 4 * h, 4 * w), dtype=torch.float32, device=self.device)
        a, d = self._dev(rgb_lo), self._dev(depth_lo)
        self._check(self.lib.gs_upsampler_forward(self.ctx, n, h, w, a.data_ptr(), d.data_ptr(),
                                                  rgb.data_ptr(), depth.data_ptr(),
                                                  _stream_ptr(torch)))
        return rgb, depth

    def up_forward_noalloc(self, rgb_lo, depth_lo, rgb_out, depth_out):
        """gs_upsampler_forward_noalloc into caller-allocated outputs: every
        tensor must already be a contiguous float32 tensor on the device of
        the right size (nothing is allocated or copied here)."""
        torch = self.torch
        n, h, w, _ = rgb_lo.shape
        shapes = ((rgb_lo, (n, h, w, 3)), (depth_lo, (n, h, w)), (rgb_out, (n, 4 * h, 4 * w, 3)),
                  (depth_out, (n, 4 * h, 4 * w)))
        for t, shp in shapes:
            if not (torch.is_tensor(t) and t.device == self.device and t.dtype == torch.float32
                    and t.is_contiguous() and tuple(t.shape) == shp):
                raise ValueError(f"expected a contiguous float32 device tensor of shape {shp}")
        self._check(self.lib.gs_upsampler_forward_noalloc(
            self.ctx, n, h, w, rgb_lo.data_ptr(), depth_lo.data_ptr(), rgb_out.data_ptr(),
            depth_out.data_ptr(), _stream_ptr(torch)))
        return rgb_out, depth_out

    def up_grads(self, rgb_lo, depth_lo, rgb_hi, depth_hi):
        n, h, w, _ = rgb_lo.shape
        tensors = [self._dev(t) for t in (rgb_lo, depth_lo, rgb_hi, depth_hi)]
        loss = ctypes.c_float()
        g = np.zeros(self.up_num_params(), np.float32)
        self._check(self.lib.gs_upsampler_grads(self.ctx, n, h, w,
                                                *[t.data_ptr() for t in tensors],
                                                ctypes.byref(loss), g.ctypes.data,
                                                _stream_ptr(self.torch)))
        return float(loss.value), g

    def up_step(self, rgb_lo, depth_lo, rgb_hi, depth_hi, lr):
        """One forward + backward + Adam step on given frames; returns the loss."""
        n, h, w, _ = rgb_lo.shape
        tensors = [self._dev(t) for t in (rgb_lo, depth_lo, rgb_hi, depth_hi)]
        loss = ctypes.c_float()
        self._check(self.lib.gs_upsampler_step(self.ctx, n, h, w, *[t.data_ptr() for t in tensors],
                                               float(lr), ctypes.byref(loss),
                                               _stream_ptr(self.torch)))
        return float(loss.value)

    def up_apply_grads(self, grads, lr):
        """One Adam update with the given gradient (parameter-vector layout)."""
        g = np.ascontiguousarray(np.asarray(grads, np.float32).reshape(-1))
        self._check(self.lib.gs_upsampler_apply_grads(self.ctx, g.ctypes.data, len(g), float(lr)))

    def up_state(self):
        """Adam state: (first moments, second moments, update count)."""
        n = self.up_num_params()
        m = np.zeros(n, np.float32)
        v = np.zeros(n, np.float32)
        step = ctypes.c_int32()
        self._check(self.lib.gs_upsampler_get_state(self.ctx, m.ctypes.data, v.ctypes.data, n,
                                                    ctypes.byref(step)))
        return m, v, int(step.value)

    def up_lr(self, step, steps, lr0, lr_min):
        return float(self.lib.gs_upsampler_lr(int(step), int(steps), float(lr0), float(lr_min)))

    def up_score(self, rgb_lo, depth_lo):
        """Fallback confidence score of low-resolution frames (device tensor [n])."""
        torch = self.torch
        n, h, w, _ = rgb_lo.shape
        a, d = self._dev(rgb_lo), self._dev(depth_lo)
        out = torch.empty(n, dtype=torch.float32, device=self.device)
        self._check(self.lib.gs_upsampler_score(self.ctx, n, h, w, a.data_ptr(), d.data_ptr(),
                                                out.data_ptr(), _stream_ptr(torch)))
        return out

    def _dev(self, a):
        """A contiguous float32 tensor on the context's device (copied when needed)."""
        torch = self.torch
        if (torch.is_tensor(a) and a.device == self.device and a.dtype == torch.float32
                and a.is_contiguous()):
            return a
        return _dev_f32(torch, a, self.device)

    def up_train(self, scene_ids, poses, intrinsics, width, height, batch=32, steps=100, lr=1e-3,
                 lr_min=0.0):
        torch = self.torch
        sids = np.ascontiguousarray(np.asarray(scene_ids, dtype=np.int32).reshape(-1))
        P = _dev_f32(torch, poses, self.device)
        K = _dev_f32(torch, intrinsics, self.device)
        o = TrainOpts(int(batch), int(steps), float(lr), float(lr_min))
        curve = np.zeros(int(steps), np.float32)
        self._check(self.lib.gs_upsampler_train(self.ctx, ctypes.byref(o), len(sids),
                                                sids.ctypes.data, P.data_ptr(), K.data_ptr(),
                                                int(width), int(height), curve.ctypes.data,
                                                _stream_ptr(torch)))
        return curve

    def render_upsampled(self, scene_ids, poses, intrinsics, width, height, threshold=float("inf"),
                         out=None, opts=None, count_fallback=True, **kw):
        """Upsampled render; returns (rgb, depth, score, n_fallback).

        With count_fallback=False the call returns before the GPU finishes
        and n_fallback is None (counting the re-rendered cameras waits)."""
        torch = self.torch
        sids = np.ascontiguousarray(np.asarray(scene_ids, dtype=np.int32).reshape(-1))
        n = len(sids)
        P, K = self._dev(poses), self._dev(intrinsics)
        if P.numel() != n * 12 or K.numel() != n * 4:
            raise ValueError("poses must be [n,3,4] and intrinsics [n,4]")
        rgb, depth, _ = out if out is not None else self.alloc_outputs(n, width, height, alpha=False)
        score = torch.empty(n, dtype=torch.float32, device=self.device)
        nf = ctypes.c_int32()
        o = opts if opts is not None else self.opts(**kw)
        self._check(self.lib.gs_render_batch_upsampled(
            self.ctx, n, sids.ctypes.data, P.data_ptr(), K.data_ptr(), int(width), int(height),
            rgb.data_ptr(), depth.data_ptr(), score.data_ptr(), float(threshold),
            ctypes.byref(nf) if count_fallback else None, ctypes.byref(o), _stream_ptr(torch)))
        return rgb, depth, score, (int(nf.value) if count_fallback else None)

    def frame_psnr(self, a, b):
        torch = self.torch
        n = a.shape[0]
        npix = a[0].numel() // 3
        out = torch.empty(n, dtype=torch.float32, device=self.device)
        self._check(self.lib.gs_frame_psnr(self.ctx, n, npix, a.contiguous().data_ptr(),
                                           b.contiguous().data_ptr(), out.data_ptr(),
                                           _stream_ptr(torch)))
        return out

    def autotune(self, scene_ids, poses, intrinsics, width, height, cache_path=None):
        torch = self.torch
        sids = np.ascontiguousarray(np.asarray(scene_ids, dtype=np.int32).reshape(-1))
        n = len(sids)
        P = _dev_f32(torch, poses, self.device)
        K = _dev_f32(torch, intrinsics, self.device)
        rgb, depth, _ = self.alloc_outputs(n, width, height, alpha=False)
        self._check(self.lib.gs_autotune(self.ctx, n, sids.ctypes.data, P.data_ptr(),
                                         K.data_ptr(), int(width), int(height), rgb.data_ptr(),
                                         depth.data_ptr(),
                                         cache_path.encode() if cache_path else None,
                                         _stream_ptr(torch)))
