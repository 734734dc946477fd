#!/usr/bin/env python3
"""Throughput of the batched Gaussian-splat renderer on one MI355X.

Workload (default): 32 synthetic terrain scenes of 50k-1M Gaussians
(7.94M in total, SH degree 3), 4096 cameras at 640x480, 128 per scene in a
shuffled scene order, RGB + expected depth in FP32. One step
renders every camera once. The paper's real scans are not available; seeded
synthetic scenes of the stated shapes stand in for them.

Timed forms
  batched  every camera in camera chunks, one launch per stage per chunk,
           captured once into a HIP graph and replayed each step (`value`)
  eager    the same kernels launched eagerly with HIP events around every
           stage (per-kernel durations for the roofline)
  plain    the per-camera kernel sequence (one camera per chunk), eager

Prints ONE JSON line (see --help). The GPU path has no fallback: the HIP
library must be built (python paper_2510_15352_amd/build.py).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "640x480 frames/s, 4096 cams: plain vs batched vs learned-upsample @PSNR"
VALU_PEAK = 256 * 4 * 16 * 2.4e9     # lane-ops/s: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
HBM_PEAK = 8.0e12                      # B/s
# Algorithmic VALU work of the path: 20 issue slots per contributing
# (pixel, Gaussian) pair (about 16 simple operations for the quadratic form,
# the clamp, the tests, the transmittance and four accumulators, plus exp at
# reduced rate) and 300 per visible (camera, Gaussian) pair for projection
# and degree-3 SH colour.
SLOTS_PER_PAIR = 20
OPS_PER_VISIBLE = 300
# VALU issue slots of every lane-pair the built raster walk issues (its ISA:
# 16 full-rate instructions plus v_exp_f32 at quarter rate); this measures
# how busy the VALUs are, waste included, not algorithmic work.
ISSUED_SLOTS = 20


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


RASTER_SOURCES = ("paper_2510_15352_amd/csrc/k_raster.hip", "paper_2510_15352_amd/csrc/gs_device.h")
TRAFFIC_PROFILE = "profiles/k_raster_workload2_hbm_traffic.md"


def gs_error():
    import paper_2510_15352_amd as gs
    return gs.GsError


def raster_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in RASTER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, cams_per_launch):
    """HBM bytes per launch of `kernel` from the committed PMC summary,
    scaled from the cameras per launch it was measured at to
    `cams_per_launch`; None when that summary is missing, has no entry for
    this kernel, or was taken on other raster sources than the ones built
    now. Returns (bytes, cameras per launch at measurement)."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None, None
    digest, entries = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- sources_sha256: "):
                digest = line.split(": ", 1)[1].strip().strip("`")
            elif line.startswith("- traffic: "):
                # - traffic: `kernel` bytes_per_launch=B cams_per_launch=C
                try:
                    name = line.split("`")[1]
                    kv = dict(t.split("=") for t in line.split("`")[2].split())
                    entries[name] = (float(kv["bytes_per_launch"]), float(kv["cams_per_launch"]))
                except (IndexError, KeyError, ValueError):
                    continue
    if digest != raster_source_digest() or kernel not in entries:
        return None, None
    b, c = entries[kernel]
    return b / c * cams_per_launch, c


def gen_workload(k):
    import scenegen
    w = scenegen.workload(k)
    t = time.time()
    scenes = [scenegen.make_scene(k, s) for s in range(w.n_scenes)]
    cams = scenegen.make_cameras(k)
    log(f"generated workload {k} ({sum(len(s['opacity']) for s in scenes)} Gaussians, "
        f"{len(cams['scene_ids'])} cameras) in {time.time() - t:.1f}s")
    return w, scenes, cams


def host_cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def time_steps(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_baseline(k, scenes, cams, W, H, budget_s, threads):
    """The FP64 oracle on a seeded sample of the same cameras."""
    import oracle
    import scenegen
    order = scenegen.camera_subset(k, len(cams["scene_ids"]), seed=777)
    done, t0 = 0, time.perf_counter()
    for c in order:
        sc = scenes[int(cams["scene_ids"][c])]
        oracle.render(sc, cams["poses"][c], cams["intrinsics"][c], W, H, threads=threads)
        done += 1
        if time.perf_counter() - t0 >= budget_s and done >= 4:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} seeded cameras of the same {len(cams['scene_ids'])}-camera "
                      f"workload, FP64 oracle, {dt:.1f}s"}


def learned_form(args, r, scenes, sids, scene_ids, P, K, W, H, n, out, ms_graph, torch):
    """Train the 4x upsampler on rendered pairs, calibrate the fallback
    threshold on held-out cameras, then time the upsampled render of the
    evaluation batch and score it against the full-resolution render."""
    import scenegen
    k = args.workload
    # the method without the network: bilinear upsampling (untrained net)
    cal = scenegen.sampled_cameras(k, args.calib_cams, seed=2)
    cal_ids = np.array([sids[i] for i in cal["scene_ids"]], np.int32)
    Pc = torch.as_tensor(cal["poses"]).cuda()
    Kc = torch.as_tensor(cal["intrinsics"]).cuda()
    full_c = r.render(cal_ids, Pc, Kc, W, H, alpha=False)
    r.up_init(0)
    up_c = r.render_upsampled(cal_ids, Pc, Kc, W, H)
    psnr_bilinear = r.frame_psnr(up_c[0], full_c[0]).cpu().numpy()
    # training on seeded pairs disjoint from calibration and evaluation
    tr = scenegen.sampled_cameras(k, args.train_pairs, seed=1)
    tr_ids = np.array([sids[i] for i in tr["scene_ids"]], np.int32)
    steps = max(1, args.train_pairs // args.train_batch)
    t = time.time()
    curve = r.up_train(tr_ids, tr["poses"], tr["intrinsics"], W, H, batch=args.train_batch,
                       steps=steps, lr=2e-3, lr_min=1e-4)
    t_train = time.time() - t
    log(f"trained upsampler: {steps} steps x {args.train_batch} pairs in {t_train:.1f}s, "
        f"loss {curve[:10].mean():.5f} -> {curve[-10:].mean():.5f}")
    # calibration: largest score below which every held-out frame reaches the target
    up_c = r.render_upsampled(cal_ids, Pc, Kc, W, H)
    psnr_c = r.frame_psnr(up_c[0], full_c[0]).cpu().numpy()
    score_c = up_c[2].cpu().numpy()
    order = np.argsort(score_c)
    bad = np.nonzero(psnr_c[order] < args.psnr_target)[0]
    if len(bad) == 0:
        thr = float("inf")
    elif bad[0] == 0:
        thr = -1.0
    else:
        thr = float(score_c[order][bad[0] - 1])
    log(f"calibration: PSNR trained mean {psnr_c.mean():.2f} dB vs bilinear "
        f"{psnr_bilinear.mean():.2f} dB; threshold {thr:.4g} accepts "
        f"{(score_c <= thr).mean():.1%} of held-out frames")
    del full_c, up_c
    # the low-resolution render gets its own tuned choice (small splats)
    if not args.no_autotune:
        r.autotune(scene_ids, P, K / 4, W // 4, H // 4)
    # timed: the evaluation batch
    uo = (torch.empty_like(out[0]), torch.empty_like(out[1]), None)

    def step_learned():
        # asynchronous: the fallback cameras are chosen on the device
        return r.render_upsampled(scene_ids, P, K, W, H, threshold=thr, out=uo,
                                  count_fallback=False)

    step_learned()
    ms = time_steps(step_learned, args.steps, torch) * 1e3
    overflowed = False
    try:
        r.status()   # raises if a timed render overflowed its instance buffers
    except gs_error() as e:
        overflowed = True
        log(f"learned form: a timed render overflowed its instance buffers ({e})")
    rgb_u, depth_u, score_u, nf = r.render_upsampled(scene_ids, P, K, W, H, threshold=thr,
                                                     out=uo)
    psnr_e = r.frame_psnr(rgb_u, out[0]).cpu().numpy()
    acc = ~(score_u.cpu().numpy() > thr)   # frames the network's output was kept for
    pa = psnr_e[acc]
    log(f"learned: {ms:.2f} ms/step, {n / ms * 1e3:.0f} frames/s, fallback {nf}/{n}; "
        f"upsampled frames: PSNR mean {pa.mean() if pa.size else float('nan'):.2f} dB")
    # fallback rate against the threshold, on the calibration frames
    curve_thr = []
    for q in (0.0, 0.1, 0.25, 0.5, 0.75, 0.9, 1.0):
        t_q = float(np.quantile(score_c, q))
        keep = score_c <= t_q
        curve_thr.append({"threshold": t_q, "fallback_rate": float(1.0 - keep.mean()),
                          "upsampled_psnr_min": float(psnr_c[keep].min()),
                          "upsampled_psnr_mean": float(psnr_c[keep].mean())})
    oracle_job = None
    if not args.no_cpu and args.oracle_frames > 0:
        oracle_job = learned_oracle_job(args, r, scene_ids, P, K, W, H, thr, torch)
    net = network_roofline(r, scene_ids, P, K, W, H, n, torch)
    held = held_out_scene_split(args, r, sids, W, H, torch) if args.held_out_split else None
    # where the step's time goes: the low-resolution render of every camera
    # (graph-replayed, as inside the form), the network, and the rest (the
    # fallback cameras' full-resolution render, scores, the head)
    lo_out = r.alloc_outputs(n, W // 4, H // 4, alpha=False)
    Klo = (K / 4).contiguous()

    def step_lo():
        r.render(scene_ids, P, Klo, W // 4, H // 4, out=lo_out, use_graph=True)

    step_lo()
    ms_lo = time_steps(step_lo, args.steps, torch) * 1e3
    r.drop_graphs()
    del lo_out
    parts = {"low_res_render": ms_lo, "network": net["ms"],
             "fallback_render_and_rest": ms - ms_lo - net["ms"]}
    log("learned form split (ms/step): " + ", ".join(f"{k} {v:.1f}" for k, v in parts.items()))
    return {"ms_per_step": ms, "frames_per_s": n / ms * 1e3, "speedup_over_batched": ms_graph / ms,
            "split_ms_per_step": parts,
            "speedup_over_plain": None,
            "fallback_rate": nf / n, "fallback_threshold": thr,
            "timed_render_overflowed": overflowed,
            "psnr_target_met_by_network": bool(pa.size and pa.min() >= args.psnr_target),
            "upsampled_frames_psnr_db": {
                "frames": int(acc.sum()),
                "mean": float(pa.mean()) if pa.size else None,
                "p5": float(np.percentile(pa, 5)) if pa.size else None,
                "min": float(pa.min()) if pa.size else None,
                "frac_ge_target": float((pa >= args.psnr_target).mean()) if pa.size else None,
                "target": args.psnr_target,
                "reference": "GPU full-resolution render of the same cameras; frames that "
                             "fall back are that render itself and are not counted"},
            "fallback_vs_threshold_calibration": curve_thr,
            "held_out_scene_split": held,
            "vs_oracle": None,   # filled in by the CPU leg
            "_oracle_job": oracle_job,
            "psnr_upsampled_only_db": {"heldout_mean_trained": float(psnr_c.mean()),
                                       "heldout_mean_bilinear": float(psnr_bilinear.mean())},
            "train": {"pairs": int(steps * args.train_batch), "batch": args.train_batch,
                      "steps": steps, "seconds": t_train, "loss_first": float(curve[:10].mean()),
                      "loss_last": float(curve[-10:].mean())},
            "network": net}


def held_out_scene_split(args, r, sids, W, H, torch):
    """Generalisation to scenes the network never saw: a second network is
    trained like the first on pairs of 24 of the 32 scenes (every fourth
    scene held out), then judged against the full-resolution render on
    cameras of the 8 held-out scenes, beside bilinear upsampling and the
    network trained on every scene. The first network's weights are put
    back afterwards."""
    import scenegen
    k = args.workload
    held = [s for s in range(len(sids)) if s % 4 == 3]
    main_w = r.up_get()
    ev = scenegen.sampled_cameras(k, args.calib_cams * 4, seed=4)
    sel = np.nonzero(np.isin(ev["scene_ids"], held))[0][:args.calib_cams // 2]
    ids = np.array([sids[i] for i in ev["scene_ids"][sel]], np.int32)
    Pe = torch.as_tensor(ev["poses"][sel]).cuda()
    Ke = torch.as_tensor(ev["intrinsics"][sel]).cuda()
    full = r.render(ids, Pe, Ke, W, H, alpha=False)

    def psnr_now():
        up = r.render_upsampled(ids, Pe, Ke, W, H)
        return r.frame_psnr(up[0], full[0]).cpu().numpy()

    p_all = psnr_now()
    r.up_init(0)
    p_bil = psnr_now()
    tr = scenegen.sampled_cameras(k, args.train_pairs * 2, seed=5)
    keep = np.nonzero(~np.isin(tr["scene_ids"], held))[0][:args.train_pairs]
    tr_ids = np.array([sids[i] for i in tr["scene_ids"][keep]], np.int32)
    steps = max(1, len(keep) // args.train_batch)
    t = time.time()
    r.up_train(tr_ids, tr["poses"][keep], tr["intrinsics"][keep], W, H, batch=args.train_batch,
               steps=steps, lr=2e-3, lr_min=1e-4)
    t_train = time.time() - t
    p_held = psnr_now()
    r.up_set(main_w)
    log(f"held-out scenes ({len(held)} scenes, {len(sel)} cameras): network trained without "
        f"them {p_held.mean():.2f} dB, trained on every scene {p_all.mean():.2f} dB, bilinear "
        f"{p_bil.mean():.2f} dB ({steps} steps in {t_train:.1f}s)")
    return {"held_out_scenes": held, "cameras": int(len(sel)), "train_steps": steps,
            "psnr_db_mean_trained_without_them": float(p_held.mean()),
            "psnr_db_p5_trained_without_them": float(np.percentile(p_held, 5)),
            "psnr_db_mean_trained_on_all": float(p_all.mean()),
            "psnr_db_mean_bilinear": float(p_bil.mean()),
            "reference": "GPU full-resolution render of the same cameras"}


def learned_oracle_job(args, r, scene_ids, P, K, W, H, thr, torch):
    """GPU side of the learned form's oracle check, on a seeded subset of the
    evaluation cameras: the upsampled render with the calibrated fallback and
    with none (the network alone), plus the low-resolution inputs and the
    weights, so that the CPU leg can run the oracle's network on them."""
    import scenegen
    pick = scenegen.camera_subset(args.workload, args.oracle_frames, seed=31)
    ids = scene_ids[pick]
    idx = torch.as_tensor(pick).cuda()
    Pp, Kp = P[idx].contiguous(), K[idx].contiguous()
    rgb, _, score, nf = r.render_upsampled(ids, Pp, Kp, W, H, threshold=thr)
    rgb_net = r.render_upsampled(ids, Pp, Kp, W, H)[0]
    m = min(args.oracle_net_frames, len(pick))
    lo_rgb, lo_depth, _ = r.render(ids[:m], Pp[:m], (Kp[:m] / 4).contiguous(), W // 4, H // 4,
                                   alpha=False)
    return {"pick": pick, "thr": thr, "nf": nf, "rgb": rgb.cpu().numpy(),
            "rgb_net": rgb_net.cpu().numpy(), "score": score.cpu().numpy(),
            "lo_rgb": lo_rgb.cpu().numpy(), "lo_depth": lo_depth.cpu().numpy(),
            "params": r.up_get()}


def learned_vs_oracle(job, k, scenes, W, H, threads):
    """CPU leg of the learned form's oracle check: PSNR and max-abs RGB error
    against the FP64 oracle render of every picked frame (the form with its
    fallback, its upsampled frames alone, and the network alone on every
    frame), and the oracle's own network on the first frames' low-resolution
    inputs, timed (frames/s) and compared with the GPU network's output."""
    import oracle
    import scenegen
    from oracle import upsampler as U
    pick, thr = job["pick"], job["thr"]
    cams = scenegen.make_cameras(k)
    t = time.time()
    psnr, err, psnr_n, err_n = [], [], [], []
    for i, c in enumerate(pick):
        sc = scenes[int(cams["scene_ids"][c])]
        ref = np.clip(oracle.render(sc, cams["poses"][c], cams["intrinsics"][c], W, H,
                                    threads=threads).rgb, 0, 1)
        for out, ps, er in ((job["rgb"], psnr, err), (job["rgb_net"], psnr_n, err_n)):
            a = np.clip(out[i].astype(np.float64), 0, 1)
            mse = float(((a - ref) ** 2).mean())
            ps.append(10.0 * np.log10(1.0 / max(mse, 1e-12)))
            er.append(float(np.abs(a - ref).max()))
    psnr, err, psnr_n, err_n = map(np.array, (psnr, err, psnr_n, err_n))
    up = ~(job["score"] > thr)
    log(f"learned vs oracle ({len(pick)} frames, {time.time() - t:.1f}s): form PSNR mean "
        f"{psnr.mean():.2f} dB, its upsampled frames "
        f"{psnr[up].mean() if up.any() else float('nan'):.2f} dB ({int(up.sum())}); network "
        f"alone {psnr_n.mean():.2f} dB (p5 {np.percentile(psnr_n, 5):.2f}), max-abs RGB "
        f"{err_n.max():.3f}")
    # the oracle's network (FP64) on the same low-resolution inputs
    x0 = U.make_input(job["lo_rgb"].astype(np.float64), job["lo_depth"].astype(np.float64))
    params = U.unflatten(job["params"].astype(np.float64))
    t0 = time.perf_counter()
    pred, _ = U.forward(x0, params)
    dt = time.perf_counter() - t0
    m = len(x0)
    gpu = job["rgb_net"][:m].astype(np.float64)
    rel_l2 = float(np.linalg.norm(gpu - pred[..., :3]) / np.linalg.norm(pred[..., :3]))
    log(f"oracle network: {m} frames in {dt:.1f}s ({m / dt:.2f} frames/s); GPU network "
        f"relative L2 {rel_l2:.2e}")
    return {"frames": int(len(pick)), "fallback_frames": int(job["nf"]),
            "psnr_db_mean": float(psnr.mean()), "psnr_db_p5": float(np.percentile(psnr, 5)),
            "max_abs_rgb": float(err.max()),
            "upsampled_frames": int(up.sum()),
            "upsampled_psnr_db_mean": float(psnr[up].mean()) if up.any() else None,
            "upsampled_max_abs_rgb": float(err[up].max()) if up.any() else None,
            "network_alone_psnr_db_mean": float(psnr_n.mean()),
            "network_alone_psnr_db_p5": float(np.percentile(psnr_n, 5)),
            "network_alone_max_abs_rgb": float(err_n.max()),
            "reference": "FP64 oracle render, RGB clamped to [0, 1]",
            "oracle_network": {"frames": m, "seconds": dt, "frames_per_s": m / dt,
                               "threads": "numpy (BLAS threads)",
                               "gpu_network_rel_l2": rel_l2}}


# multiply-accumulates per low-resolution pixel of the 4x upsampler: 3x3
# convolutions 4->32, 32->32, 32->32, 32->64
UP_MACS_PER_PIXEL = 9 * (4 * 32 + 32 * 32 + 32 * 32 + 32 * 64)
MFMA_BF16_PEAK_TFLOPS = 2500.0


def network_roofline(r, scene_ids, P, K, W, H, n, torch):
    """The upsampler network alone on the batch's low-resolution frames:
    HIP-event time, algorithmic TFLOP/s against the dense BF16 MFMA peak,
    and its algorithmic HBM traffic (16 B per low-resolution input pixel,
    16 B per full-resolution output pixel)."""
    h, w = H // 4, W // 4
    lo_rgb, lo_depth, _ = r.render(scene_ids, P, K / 4, w, h, alpha=False)
    r.up_forward(lo_rgb, lo_depth)  # outputs allocated once, then reused by the caching allocator
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        r.up_forward(lo_rgb, lo_depth)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    px = n * h * w
    tflop = 2.0 * UP_MACS_PER_PIXEL * px / 1e12
    gbytes = (16 * px + 16 * px * 16) / 1e9
    tflops = tflop / (ms / 1e3)
    log(f"network alone: {ms:.2f} ms for {n} frames of {w}x{h}: {tflops:.0f} TFLOP/s "
        f"({tflops / MFMA_BF16_PEAK_TFLOPS:.3f} of the BF16 MFMA peak), "
        f"{gbytes / (ms / 1e3):.0f} GB/s algorithmic HBM traffic")
    return {"ms": ms, "frames": n, "low_res": [w, h], "bound": "mfma",
            "algorithmic_tflop": tflop, "achieved_tflops": tflops,
            "peak_tflops": MFMA_BF16_PEAK_TFLOPS, "frac": tflops / MFMA_BF16_PEAK_TFLOPS,
            "hbm_algorithmic_GB": gbytes, "hbm_GB_per_s": gbytes / (ms / 1e3),
            "hbm_frac": gbytes / (ms / 1e3) / 8000.0}


def stress_leg(args, r, torch):
    """The stress workload (one 3M-Gaussian scene, 8192 cameras at 320x240)
    over a few consecutive sim steps: every camera advances along its
    trajectory each step, the step's poses are copied into the buffer the
    captured graph reads and the graph is replayed (every stage recomputed).
    Fixed choice (16x8 tiles, LDS batch 64, 64-camera chunks: the
    autotuner's pick for this workload), so the leg needs no tuning time. Also the pair counts of one
    step (instrumented raster)."""
    import scenegen
    k = 4
    w = scenegen.workload(k)
    t = time.time()
    sc = scenegen.make_scene(k, 0)
    traj = scenegen.camera_steps(k, args.stress_steps)
    log(f"stress leg: generated {len(sc['opacity'])} Gaussians and {args.stress_steps} steps of "
        f"{w.n_cams} cameras in {time.time() - t:.1f}s")
    sid = r.upload_scene(sc)
    n, W, H = w.n_cams, w.width, w.height
    ids = np.full(n, sid, np.int32)
    trajd = torch.as_tensor(traj["poses"]).cuda()
    P = trajd[0].clone()
    K = torch.as_tensor(traj["intrinsics"]).cuda()
    out = r.alloc_outputs(n, W, H, alpha=False)
    kw = dict(tile=(16, 8), lds_batch=64, persistent=0, chunk_cams=64)

    def step(i):
        P.copy_(trajd[i % args.stress_steps])
        r.render(ids, P, K, W, H, out=out, use_graph=True, **kw)

    for i in range(2):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.stress_steps):
        step(i)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.stress_steps * 1e3
    st = r.stats()
    P.copy_(trajd[0])
    r.render(ids, P, K, W, H, out=out, count_pairs=True, **kw)
    sc_ = r.stats()
    pairs, evals, issued = sc_["pairs_contrib"], sc_["pairs_evaluated"], sc_["pairs_issued"]
    b_g = 44 + 12 * (w.sh_degree + 1) ** 2
    alg = 16.0 * W * H * n + float(len(sc["opacity"])) * b_g + 24.0 * float(st["instances"])
    log(f"stress leg: {ms:.1f} ms/step over {args.stress_steps} consecutive steps, "
        f"{n / ms * 1e3:.0f} frames/s; evaluated/contributing {evals / max(pairs, 1):.2f}, "
        f"issued/contributing {issued / max(pairs, 1):.2f}")
    r.drop_graphs()
    r.release_scene(sid)
    del out, trajd
    return {"workload": w.name, "steps": args.stress_steps, "ms_per_step": ms,
            "frames_per_s": n / ms * 1e3, "form": "batched, hipGraph replay, poses advanced "
            "every sim step", "choice": {k_: st[k_] for k_ in ("tile_w", "tile_h", "lds_batch",
                                                                "chunk_cams", "persistent")},
            "pairs_per_step": pairs, "eval_over_contrib": evals / max(pairs, 1),
            "issued_over_contrib": issued / max(pairs, 1),
            "hbm_algorithmic_GB_per_s": alg / (ms * 1e-3) / 1e9}


def backward_leg(args, r, torch):
    """The backward pass (gradients of RGB, depth and alpha with respect to
    every Gaussian parameter) over the 64 cameras of the 200k-Gaussian SH-3
    terrain scene at 640x480, random upstream gradients; each call waits
    for its result."""
    import scenegen
    sc = scenegen.make_scene(1)
    cams = scenegen.make_cameras(1)
    sid = r.upload_scene(sc)
    n, W, H = len(cams["poses"]), cams["width"], cams["height"]
    P = torch.as_tensor(cams["poses"]).cuda()
    K = torch.as_tensor(cams["intrinsics"]).cuda()
    g = torch.Generator(device="cuda").manual_seed(5)
    gr = torch.randn((n, H, W, 3), device="cuda", generator=g)
    gd = 0.1 * torch.randn((n, H, W), device="cuda", generator=g)
    ga = torch.randn((n, H, W), device="cuda", generator=g)
    r.render_backward(sid, P, K, W, H, gr, gd, ga)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        r.render_backward(sid, P, K, W, H, gr, gd, ga)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    r.render([sid] * n, P, K, W, H, use_graph=False)
    ms_fwd = time_steps(lambda: r.render([sid] * n, P, K, W, H), 3, torch) * 1e3
    r.release_scene(sid)
    log(f"backward: {ms:.1f} ms for {n} cameras of 640x480 ({n / ms * 1e3:.0f} frames/s), "
        f"forward {ms_fwd:.1f} ms")
    return {"workload": "slab200k_sh3_64cams_640x480", "cams": n, "ms": ms,
            "frames_per_s": n / ms * 1e3, "forward_ms": ms_fwd,
            "upstream": "random normal dL/dRGB, 0.1 x normal dL/ddepth, normal dL/dalpha"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 5; 100 consecutive sim steps for workload 4)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 4])
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--autotune-cache", default=None, metavar="PATH",
                    help="autotune cache file (JSON lines): a result for this GPU and workload "
                         "is read back instead of tuning, a new one appended")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (tile shape, LDS batch, chunk size, persistence) "
                         "and use the library's default choice")
    ap.add_argument("--only-batched", action="store_true",
                    help="time only the graph-replayed batched form (for profiling)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-upsample form")
    ap.add_argument("--choice", type=int, nargs=4, default=None, metavar=("TW", "TH", "B", "C"),
                    help="render with tile TWxTH, LDS batch B, C cameras per chunk (grid "
                         "raster) instead of the autotuner's choice (for profiling)")
    ap.add_argument("--form", type=int, default=0, choices=[0, 1],
                    help="raster form with --choice: 0 grid, 1 persistent work queue")
    ap.add_argument("--train-pairs", type=int, default=100_000)
    ap.add_argument("--train-batch", type=int, default=64)
    ap.add_argument("--calib-cams", type=int, default=512)
    ap.add_argument("--psnr-target", type=float, default=35.0)
    ap.add_argument("--oracle-frames", type=int, default=128,
                    help="evaluation frames of the learned form checked against the FP64 oracle")
    ap.add_argument("--no-held-out-split", dest="held_out_split", action="store_false",
                    help="skip training a second upsampler without 8 of the scenes")
    ap.add_argument("--oracle-net-frames", type=int, default=32,
                    help="of those, frames the oracle's FP64 network runs on (timed)")
    ap.add_argument("--stress-steps", type=int, default=10,
                    help="consecutive sim steps of the stress workload timed beside the default "
                         "workload (0: skip that leg)")
    ap.add_argument("--no-backward", action="store_true",
                    help="skip timing the backward pass")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device a few times and exit (reference "
                         "kernel for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}))
        return
    if args.steps is None:
        args.steps = 100 if args.workload == 4 else 5
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(cameras shard across GPUs with no exchange between them, so one GPU's "
              "share at its real shape is what this measures)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2510_15352_amd as gs
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    w, scenes, cams = gen_workload(args.workload)
    W, H = cams["width"], cams["height"]
    n = len(cams["scene_ids"])
    r = gs.Renderer(0)
    t = time.time()
    sids = [r.upload_scene(s) for s in scenes]
    torch.cuda.synchronize()
    log(f"uploaded {len(sids)} scenes in {time.time() - t:.1f}s")
    scene_ids = np.array([sids[i] for i in cams["scene_ids"]], np.int32)
    P = torch.as_tensor(cams["poses"]).cuda()
    K = torch.as_tensor(cams["intrinsics"]).cuda()
    # the metric's outputs: RGB + expected depth (no alpha)
    out = r.alloc_outputs(n, W, H, alpha=False)
    tuned = None
    choice_kw = {}
    if args.choice:
        tw, th, b, c = args.choice
        choice_kw = dict(tile=(tw, th), lds_batch=b, chunk_cams=c, persistent=args.form)
    if not args.no_autotune and not args.choice:
        t = time.time()
        r.autotune(scene_ids, cams["poses"], cams["intrinsics"], W, H,
                   cache_path=args.autotune_cache)
        tuned = True
        log(f"autotune done in {time.time() - t:.1f}s")

    # batched + graph: the headline form. Workload 4 advances every camera
    # along its trajectory each sim step: the step's poses are copied into
    # the buffer the captured graph reads, then the graph is replayed (every
    # stage, sorts included, recomputed).
    traj = None
    if w.steps > 1:
        import scenegen
        t = time.time()
        traj = torch.as_tensor(scenegen.camera_steps(args.workload, w.steps)["poses"]).cuda()
        log(f"{w.steps} steps of trajectories in {time.time() - t:.1f}s")
    sim_step = [0]

    def step_graph():
        if traj is not None:
            P.copy_(traj[sim_step[0] % w.steps])
            sim_step[0] += 1
        r.render(scene_ids, P, K, W, H, out=out, use_graph=True, **choice_kw)

    for i in range(args.warmup):
        step_graph()
        log(f"warmup step {i} done")
    sim_step[0] = 0
    ms_graph = time_steps(step_graph, args.steps, torch) * 1e3
    st_graph = r.stats()
    log(f"batched+graph: {ms_graph:.2f} ms/step, {n / ms_graph * 1e3:.0f} frames/s")
    if traj is not None:
        P.copy_(traj[0])
    forms = {"batched": {"ms_per_step": ms_graph, "frames_per_s": n / ms_graph * 1e3,
                         "choice": {k: st_graph[k] for k in ("tile_w", "tile_h", "lds_batch",
                                                              "chunk_cams", "persistent")}}}
    roofline = None
    if not args.only_batched:
        # eager batched with HIP events per stage (same kernels, same inputs)
        stage_ms = {}
        stage_n = {}

        def step_eager():
            r.render(scene_ids, P, K, W, H, out=out, timing=True, **choice_kw)
            s = r.stats()
            for k, v in s["stage_ms"].items():
                stage_ms[k] = stage_ms.get(k, 0.0) + v
                stage_n[k] = stage_n.get(k, 0) + s["stage_launches"][k]

        step_eager()
        stage_ms.clear()
        stage_n.clear()
        # the per-stage split needs only a few steps (the poses stay at the
        # first sim step of a trajectory workload)
        eager_steps = min(args.steps, 5)
        ms_eager = time_steps(step_eager, eager_steps, torch) * 1e3
        per_step = {k: v / eager_steps for k, v in stage_ms.items()}
        log("eager stages (ms/step): " + ", ".join(f"{k} {v:.2f}" for k, v in per_step.items()))
        forms["batched_eager"] = {"ms_per_step": ms_eager, "frames_per_s": n / ms_eager * 1e3,
                                  "stage_ms_per_step": per_step}
        # pair counts (instrumented raster, untimed)
        r.render(scene_ids, P, K, W, H, out=out, count_pairs=True, **choice_kw)
        sc = r.stats()
        pairs, evals, issued = sc["pairs_contrib"], sc["pairs_evaluated"], sc["pairs_issued"]
        dom = max(per_step, key=per_step.get)
        raster_launch_ms = stage_ms["raster"] / max(stage_n["raster"], 1)
        pairs_per_launch = pairs / max(stage_n["raster"] / eager_steps, 1)
        achieved = pairs_per_launch * SLOTS_PER_PAIR / (raster_launch_ms * 1e-3)
        kname = "gs::%s<%d, %d, %d>" % (
            {0: "k_raster", 1: "k_raster_persistent"}[st_graph["persistent"]],
            st_graph["tile_w"], st_graph["tile_h"], st_graph["lds_batch"])
        launches = stage_n["raster"] / eager_steps
        traffic, traffic_cams = measured_traffic(kname, n / max(launches, 1))
        roofline = {"bound": "alu", "kernel": kname, "achieved": achieved / 1e12,
                    "peak": VALU_PEAK / 1e12, "unit": "T VALU lane-ops/s",
                    "frac": achieved / VALU_PEAK, "traffic": traffic,
                    "traffic_unit": "HBM bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, "
                                    "copy-calibrated; measured at traffic_cams_per_launch "
                                    "cameras per launch, scaled to this launch's cameras)",
                    "traffic_cams_per_launch": traffic_cams,
                    "avg_launch_ms": raster_launch_ms,
                    "launches_per_step": stage_n["raster"] / eager_steps,
                    "pairs_per_step": pairs, "evaluated_pairs_per_step": evals,
                    "eval_over_contrib": evals / max(pairs, 1),
                    "issued_lanes_per_step": issued, "issued_over_contrib": issued / max(pairs, 1),
                    # the same roofline over every lane-pair the walk issues
                    # (17 VALU instructions, v_exp_f32 at quarter rate: 20
                    # slots): how busy the VALUs are, waste included
                    "issued_frac": (issued / max(stage_n["raster"] / eager_steps, 1)) * ISSUED_SLOTS
                                   / (raster_launch_ms * 1e-3) / VALU_PEAK,
                    "slots_per_pair": SLOTS_PER_PAIR, "dominant_stage": dom,
                    "visible_pairs_per_step": sc["visible"], "instances_per_step": sc["instances"]}
        # measured peaks beside the published ones
        fma_rate, exp_rate, copy_rate = (r.peak_probe(k) for k in (0, 1, 2))
        roofline["measured_peak"] = {
            "fma_lane_ops_per_s": fma_rate, "exp_lane_ops_per_s": exp_rate,
            "copy_bytes_per_s": copy_rate,
            "frac": achieved / fma_rate,
            "issued_frac": roofline["issued_frac"] * VALU_PEAK / fma_rate}
        log(f"measured peaks: FMA {fma_rate / 1e12:.1f} T lane-ops/s, exp {exp_rate / 1e12:.1f} T, "
            f"copy {copy_rate / 1e12:.2f} TB/s")
        log(f"raster: {raster_launch_ms:.3f} ms/launch, pairs {pairs:.3e}, evaluated {evals:.3e}, "
            f"issued lanes {issued:.3e}, frac {roofline['frac']:.3f}, "
            f"issued frac {roofline['issued_frac']:.3f}")
        # plain form: per-camera kernel sequence
        if args.plain_steps > 0:
            def step_plain():
                r.render(scene_ids, P, K, W, H, out=out, mode="plain")
            step_plain()
            ms_plain = time_steps(step_plain, args.plain_steps, torch) * 1e3
            forms["plain"] = {"ms_per_step": ms_plain, "frames_per_s": n / ms_plain * 1e3}
            log(f"plain: {ms_plain:.1f} ms/step")
            forms["batched"]["speedup_over_plain"] = ms_plain / ms_graph

    if not args.only_batched and not args.no_learned and args.workload == 2:
        forms["learned"] = learned_form(args, r, scenes, sids, scene_ids, P, K, W, H, n, out,
                                        ms_graph, torch)
        if "plain" in forms:
            forms["learned"]["speedup_over_plain"] = (forms["plain"]["ms_per_step"] /
                                                      forms["learned"]["ms_per_step"])

    if not args.only_batched and args.workload == 2 and args.stress_steps > 0:
        forms["stress_workload4"] = stress_leg(args, r, torch)
    if not args.only_batched and not args.no_backward and args.workload == 2:
        forms["backward"] = backward_leg(args, r, torch)

    # the CPU leg: the oracle timed on a sample of the workload (the
    # baseline) and the learned form's frames judged by the oracle
    cpu = None
    job = forms.get("learned", {}).pop("_oracle_job", None)
    if not args.no_cpu:
        threads = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "64")))
        cpu = cpu_baseline(args.workload, scenes, cams, W, H, args.cpu_seconds, threads)
        cpu["host_cpus"] = os.cpu_count()
        cpu["cpu_model"] = host_cpu_model()
        log(f"cpu oracle: {cpu['value']:.3f} frames/s on {threads} threads "
            f"({cpu['cpu_model']}, {cpu['host_cpus']} CPUs on the host)")
        if job is not None:
            forms["learned"]["vs_oracle"] = learned_vs_oracle(job, args.workload, scenes, W, H,
                                                              threads)
    del job

    # algorithmic HBM bytes of one step: outputs (RGB + depth [+ alpha], FP32),
    # every scene's parameters read once, 24 B per tile instance
    b_g = 44 + 12 * (w.sh_degree + 1) ** 2
    px_bytes = 12 + 4 + (4 if out[2] is not None else 0)
    alg_bytes = (float(px_bytes) * W * H * n + float(sum(len(s["opacity"]) for s in scenes)) * b_g
                 + 24.0 * float(st_graph["instances"]))
    hbm = {"algorithmic_bytes_per_step": alg_bytes,
           "GB_per_s": alg_bytes / (ms_graph * 1e-3) / 1e9,
           "frac_of_peak": alg_bytes / (ms_graph * 1e-3) / HBM_PEAK,
           "model": f"{px_bytes} B/pixel out + {b_g} B per Gaussian once + 24 B per instance",
           "instances_per_step": st_graph["instances"], "visible_per_step": st_graph["visible"]}
    log(f"algorithmic HBM traffic {alg_bytes / 1e9:.2f} GB/step = {hbm['GB_per_s']:.0f} GB/s")

    if roofline is not None:
        # the whole path against its roofline: VALU work of the raster and
        # the projection, HBM bytes of the step (no MFMA on this path)
        t_valu = (SLOTS_PER_PAIR * float(roofline["pairs_per_step"]) +
                  OPS_PER_VISIBLE * float(st_graph["visible"])) / VALU_PEAK
        t_hbm = alg_bytes / HBM_PEAK
        t_roof = max(t_valu, t_hbm)
        roofline["path"] = {
            "t_valu_ms": t_valu * 1e3, "t_hbm_ms": t_hbm * 1e3, "t_mfma_ms": 0.0,
            "bound": "valu" if t_valu >= t_hbm else "hbm",
            "roofline_frames_per_s": n / t_roof, "achieved_frames_per_s": n / (ms_graph * 1e-3),
            "model": f"{SLOTS_PER_PAIR} VALU slots per contributing pair + {OPS_PER_VISIBLE} per "
                     "visible (camera, Gaussian) pair at 39.3 T lane-ops/s; algorithmic bytes "
                     "at 8 TB/s"}
        roofline["path_frac"] = t_roof / (ms_graph * 1e-3)
        log(f"path roofline: VALU {t_valu * 1e3:.2f} ms, HBM {t_hbm * 1e3:.2f} ms per step; "
            f"achieved {ms_graph:.2f} ms -> path_frac {roofline['path_frac']:.3f}")

    line = {
        "metric": METRIC, "value": n / ms_graph * 1e3, "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_graph,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "cams": n, "width": W, "height": H,
                   "scenes": w.n_scenes, "gaussians": int(sum(len(s["opacity"]) for s in scenes)),
                   "sh_degree": w.sh_degree, "sim_steps": w.steps,
                   "form": "batched, hipGraph replay" + (
                       ", poses advanced every sim step" if w.steps > 1 else "")},
        "forms": forms, "roofline": roofline, "cpu_baseline": cpu, "hbm_algorithmic": hbm,
    }
    # the choice the timed renders used (the autotuner's pick unless
    # --no-autotune)
    line["config"]["choice"] = dict(forms["batched"]["choice"], autotuned=bool(tuned))
    print(json.dumps(line), flush=True)
    r.close()


if __name__ == "__main__":
    main()
