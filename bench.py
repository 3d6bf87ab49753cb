#!/usr/bin/env python3
"""Benchmark of the VaFR hot path on one MI355X.

One step = one binocular frame at 7680 x 4320 per eye (100 x 100 degree field
of view): for each eye, shade the constant-size LP buffer (one primary ray and
one shadow ray per texel against a 4,521,984-triangle scene) and inverse-map it
onto the display.  The gaze of frame f comes from a seeded fixation/saccade
trace.  The same GPU also runs the full-resolution ray cast and the LMFR(1.8),
LaFR(1.8) and LaFR(2.2) mappings for the speed-ups.  Inputs are synthetic and already resident in HBM
when timing starts.

Prints ONE JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

W, H = 7680, 4320
SCENE = "terrain4m"
FRAME_BUDGET_MS = 11.1    # one refresh at 90 Hz
# Peak figures of the MI355X (published): HBM3E bandwidth, and the VALU lane
# issue rate = 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one non-packed FP32
# operation per lane per clock; 157.3 TFLOP/s counts packed FMA as 4 flops).
HBM_PEAK_GBS = 8000.0
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4

# FP32 operations of one unit of traversal work, counted from the arithmetic
# the traversal performs:
#  - one node visit tests four child boxes.  Algorithmic part: per node 3
#    FMAs and 3 multiplies (distance to the node origin, scale / d); per
#    child 6 FMAs for the slab distances (the benchmark's eyes are within
#    the range where this form is conservative), 4 min/max to combine axes
#    and clamp, 1 multiply (conservative exit) and 1 compare; then 3 adds
#    (hit count), 4 selects (misses sort last) and a 5-exchange sorting
#    network of (distance, reference) pairs, 1 compare + 4 selects each
#    -> 6 + 4 * 12 + 3 + 4 + 25 = 86.
#    Node-format part (the library's own 8-bit quantised node): 6 selects
#    (entry / exit plane codes by the ray's direction signs) and per child 6
#    byte-to-float code conversions -> 6 + 4 * 6 = 30.  These are counted
#    separately: a node format that stored FP32 planes would not need them.
#  - one watertight ray/triangle test: 9 subtractions (vertices - origin),
#    6 FMAs (shear), 6 multiplies + 3 subtractions (edge functions), 2 adds
#    (det), 3 multiplies (z scaling), 3 multiplies + 2 adds (T), 1 division,
#    4 compares -> 39
#  - ray set-up: 3 reciprocals, 3 multiplies (o/d), 3 divisions, 8
#    compares/selects -> 17
OPS_NODE = 86
OPS_NODE_FORMAT = 30
OPS_TRI = 39
OPS_RAY = 17
# frames of the comparison legs (full resolution, LMFR, LaFR, layouts, ...)
# and of the two-frames-in-flight leg, whatever --steps says
MIN_COMPARE_FRAMES = 20
MIN_PIPELINED_FRAMES = 100


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(x, q):
    return float(np.percentile(np.asarray(x, np.float64), q))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("trace.hip", "reconstruct.hip"):
        with open(os.path.join(ROOT, "paper_2503_23410_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(kind):
    """SQ counter summary of a kernel (VALU issue per SIMD per clock, active
    lanes, resident waves) measured with rocprofv3 --pmc for the current
    kernel sources, or None."""
    path = os.path.join(ROOT, "profiles", "pmc_sq.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(kind)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return {k: e[k] for k in ("valu_per_simd_clock", "active_lane_frac", "resident_waves_per_simd",
                              "wait_frac") if k in e}


def load_traffic(kind):
    """HBM traffic per launch measured with rocprofv3 --pmc (FETCH_SIZE,
    WRITE_SIZE) for the current kernel sources, or None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(kind)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=900,
                    help="timed binocular VaFR frames (900 = 10 s of the 90 Hz gaze trace)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--compare-steps", type=int, default=0,
                    help="frames for the full-resolution and LMFR comparisons (default: steps/20, >= 3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip full-resolution and LMFR runs")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="duration of the served 8-headset workload per server configuration (0: skip)")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the two-frames-in-flight leg (kernel traces of the one-at-a-time frames)")
    ap.add_argument("--profile-summary", metavar="DIR",
                    help="summarise rocprofv3 output under DIR into profiles/ and exit (no GPU use)")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(views would be sharded across GPUs, each holding a replica of the scene, with no exchange).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_23410_amd import inputs as I
    from paper_2503_23410_amd import vafr as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    V.load()
    steps, warm = args.steps, args.warmup
    csteps = args.compare_steps or max(MIN_COMPARE_FRAMES, steps // 20)

    t = time.time()
    verts, tris = I.make_scene(SCENE)
    log(f"scene {SCENE}: {tris.shape[0]} triangles generated in {time.time() - t:.1f}s")
    scene = V.Scene(verts, tris)
    info = scene.info()
    log(f"BVH: {info['n_nodes']} nodes, depth {info['max_depth']}, built in {info['build_ms']:.0f} ms, "
        f"{info['device_bytes'] / 1e6:.0f} MB on device")
    disp = V.display(W, H, I.FOV)
    L = V.Layout.vafr(disp)
    LM = V.Layout.lmfr(disp, 1.8, 4.0)
    cams = [V.camera(c) for c in I.binocular_cameras()]
    sh = V.shading()
    trace = I.gaze_trace(warm + max(steps, csteps, MIN_PIPELINED_FRAMES), W, H, seed=30)
    gazes = [V.gaze(float(x), float(y)) for x, y in trace]

    lp = [torch.empty((L.n_texels, 4), device="cuda", dtype=torch.float32) for _ in range(2)]
    img = [torch.empty((H * W, 4), device="cuda", dtype=torch.float32) for _ in range(2)]
    stream = torch.cuda.current_stream()

    def vafr_frame(f, ev=None):
        g = gazes[f]
        for e in range(2):
            if ev is not None:
                ev[2 * e].record(stream)
            V.vafr_shade_lp(scene, cams[e], g, sh, L, lp[e], None, stream)
            if ev is not None:
                ev[2 * e + 1].record(stream)
            V.vafr_reconstruct(L, g, lp[e], img[e], stream)
        if ev is not None:
            ev[4].record(stream)

    # ------------------------------------------------------------ VaFR
    # (a) plain per-view calls: shade + reconstruct per eye
    for f in range(warm):
        vafr_frame(f)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(steps):
        vafr_frame(warm + f, evs[f])
    torch.cuda.synchronize()
    wall_plain = time.perf_counter() - t0
    frame_ms_plain, trace_ms, recon_ms = [], [], []
    for ev in evs:
        frame_ms_plain.append(ev[0].elapsed_time(ev[4]))
        trace_ms += [ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])]
        recon_ms += [ev[1].elapsed_time(ev[2]), ev[3].elapsed_time(ev[4])]
    fps_plain = steps / wall_plain
    log(f"VaFR per-view calls: {fps_plain:.1f} frames/s, frame p50 {percentile(frame_ms_plain, 50):.3f} ms "
        f"p99 {percentile(frame_ms_plain, 99):.3f} ms; trace {np.mean(trace_ms):.3f} ms/eye, "
        f"reconstruct {np.mean(recon_ms):.3f} ms/eye")

    # (b) batched frame: both eyes in one traversal + one reconstruction
    # launch, replayed from a hipGraph, launch shape autotuned
    batch = V.Batch(2)

    def bviews(f):
        g = gazes[f]
        return [V.view(V.VAFR_VIEW_VAFR, scene, cams[e], g, sh, layout=L, lp_rgba=lp[e], img_rgba=img[e])
                for e in range(2)]

    tuned = batch.autotune(bviews(0), reps=5, stream=stream)
    batch.set_profiling(False)
    for f in range(warm):
        batch.run(bviews(f), stream)
    torch.cuda.synchronize()
    bev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    t0 = time.perf_counter()
    for f in range(steps):
        bev[f][0].record(stream)
        batch.run(bviews(warm + f), stream)
        bev[f][1].record(stream)
    torch.cuda.synchronize()
    wall_batch = time.perf_counter() - t0
    frame_ms_batch = [ev[0].elapsed_time(ev[1]) for ev in bev]
    # stage times from event nodes inside the graph (read without host
    # syncs), in a pass of their own over the same frames
    batch.set_profiling(True)
    for f in range(min(steps, 300)):
        batch.run(bviews(warm + f), stream)
    torch.cuda.synchronize()
    (b_upload_ms, b_trace_ms, b_recon_ms), b_frames = batch.stage_ms()
    fps_batch = steps / wall_batch
    log(f"VaFR batched ({tuned}): {fps_batch:.1f} frames/s, frame p50 {percentile(frame_ms_batch, 50):.3f} ms "
        f"p99 {percentile(frame_ms_batch, 99):.3f} ms; stages over {b_frames} frames: upload {b_upload_ms:.4f} ms, "
        f"trace {b_trace_ms:.4f} ms, reconstruct {b_recon_ms:.4f} ms (both eyes)")
    if fps_batch >= fps_plain:
        fps, wall, frame_ms, path = fps_batch, wall_batch, frame_ms_batch, "batched"
    else:
        fps, wall, frame_ms, path = fps_plain, wall_plain, frame_ms_plain, "per-view"

    # work counts of the traversal (one frame, both eyes, gaze of frame warm)
    counters = torch.zeros(4, device="cuda", dtype=torch.int64)
    for e in range(2):
        V.vafr_count_work(scene, cams[e], gazes[warm], sh, L, counters, stream)
    torch.cuda.synchronize()
    n_prim, n_shadow, n_nodes, n_tri = [int(x) for x in counters.cpu()]
    ops_frame = OPS_NODE * n_nodes + OPS_TRI * n_tri + OPS_RAY * (n_prim + n_shadow)
    ops_frame_fmt = ops_frame + OPS_NODE_FORMAT * n_nodes
    recon_bytes_frame = 2 * (W * H * 16 + L.n_texels * 16)
    if path == "batched":
        # one traversal launch and one reconstruction launch per frame
        k_trace, k_recon = "k_trace_batch", "k_recon_batch"
        ops_per_launch, trace_s = ops_frame, b_trace_ms / 1e3
        ops_fmt_per_launch = ops_frame_fmt
        recon_bytes, recon_s = recon_bytes_frame, b_recon_ms / 1e3
    else:
        k_trace, k_recon = "k_trace", "k_recon"
        ops_per_launch, trace_s = ops_frame / 2.0, float(np.mean(trace_ms)) / 1e3
        ops_fmt_per_launch = ops_frame_fmt / 2.0
        recon_bytes, recon_s = recon_bytes_frame / 2.0, float(np.mean(recon_ms)) / 1e3
    achieved_gops = ops_per_launch / trace_s / 1e9
    rays_per_s = (n_prim + n_shadow) / (2.0 if path != "batched" else 1.0) / trace_s
    recon_gbs = recon_bytes / recon_s / 1e9
    log(f"work per eye: {n_prim // 2} primary + {n_shadow // 2} shadow rays, {n_nodes / (n_prim + n_shadow):.1f} "
        f"node visits and {n_tri / (n_prim + n_shadow):.2f} triangle tests per ray; "
        f"{rays_per_s / 1e9:.2f} Grays/s; reconstruct {recon_gbs:.0f} GB/s")

    out = {}
    # two frames in flight: alternate batches on two streams with double
    # buffers, so one frame's reconstruction overlaps the next one's
    # traversal (throughput up, per-frame latency up)
    if not args.no_pipelined:
        out["pipelined"] = pipelined_frames(torch, V, scene, cams, sh, L, gazes, warm,
                                            max(MIN_PIPELINED_FRAMES, min(steps, 600)), tuned)
    # ------------------------------------------------------------ comparisons
    if not args.no_compare:
        # full resolution: one primary + shadow ray per display pixel, per eye
        def full_frame(f, ev=None):
            if ev is not None:
                ev[0].record(stream)
            for e in range(2):
                V.full_shade(scene, cams[e], disp, sh, img[e], None, stream)
            if ev is not None:
                ev[1].record(stream)

        full_frame(0)
        torch.cuda.synchronize()
        fev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(csteps)]
        t0 = time.perf_counter()
        for f in range(csteps):
            full_frame(f, fev[f])
        torch.cuda.synchronize()
        full_fps = csteps / (time.perf_counter() - t0)
        full_ms = [ev[0].elapsed_time(ev[1]) for ev in fev]
        log(f"full resolution: {full_fps:.2f} frames/s (frame {np.mean(full_ms):.2f} ms)")
        # dense log-polar comparisons: LMFR(1.8), LaFR(1.8), LaFR(2.2)
        def dense_fps(layout, shade, recon):
            lpl = torch.empty((layout.n_texels, 4), device="cuda", dtype=torch.float32)

            def frame(f, ev=None):
                g = gazes[warm + f]
                if ev is not None:
                    ev[0].record(stream)
                for e in range(2):
                    shade(scene, cams[e], g, sh, layout, lpl, None, stream)
                    recon(layout, g, lpl, img[e], stream)
                if ev is not None:
                    ev[1].record(stream)

            frame(0)
            torch.cuda.synchronize()
            evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(csteps)]
            t0 = time.perf_counter()
            for f in range(csteps):
                frame(f, evs[f])
            torch.cuda.synchronize()
            rate = csteps / (time.perf_counter() - t0)
            return rate, float(np.mean([ev[0].elapsed_time(ev[1]) for ev in evs]))

        lmfr_fps, lmfr_ms = dense_fps(LM, V.lmfr_shade_lp, V.lmfr_reconstruct)
        log(f"LMFR(1.8): {lmfr_fps:.2f} frames/s (frame {lmfr_ms:.2f} ms)")
        lafr = {}
        for delta in (1.8, 2.2):
            LA = V.Layout.lafr(disp, delta)
            rate, ms = dense_fps(LA, V.lafr_shade_lp, V.lafr_reconstruct)
            log(f"LaFR({delta}): {rate:.2f} frames/s (frame {ms:.2f} ms), {LA.n_texels} texels per eye")
            lafr[str(delta)] = {"fps": round(rate, 3), "frame_ms": round(ms, 3), "texels_per_eye": LA.n_texels,
                                "speedup": round(fps / rate, 2)}
            LA.close()
        out["lafr"] = lafr
        out.update({
            "fullres_fps": round(full_fps, 3), "fullres_frame_ms": round(float(np.mean(full_ms)), 3),
            "lmfr_fps": round(lmfr_fps, 3), "lmfr_frame_ms": round(lmfr_ms, 3),
            "speedup_vs_fullres": round(fps / full_fps, 2), "speedup_vs_lmfr": round(fps / lmfr_fps, 2),
            "speedup_vs_lafr": lafr["1.8"]["speedup"],
            "fullres_grays_per_s": round(2 * 2 * W * H * full_fps / 1e9, 3),
            "compare_frames": csteps,
        })

    # ------------------------------------------------------------ LP anti-aliasing
    if not args.no_compare:
        out["fxaa"] = fxaa_bench(torch, V, scene, cams, sh, L, gazes[warm:], max(20, csteps))

    # ------------------------------------------------------------ reprojection
    if not args.no_compare:
        out["rep"] = rep_bench(torch, V, scene, cams, sh, L, gazes[warm:], max(20, csteps))

    # ------------------------------------------------------------ 16 views
    if not args.no_compare:
        out["batch16"] = batch16(torch, V, I, scene, sh, csteps)
        out["layouts"] = layout_variants(torch, V, I, scene, sh, cams, gazes, warm, max(20, csteps), tuned)
        out["resolutions"] = resolution_sweep(torch, V, I, scene, sh, cams, max(60, 10 * csteps), max(2, csteps),
                                              tuned)

    # ------------------------------------------------------------ serving
    if args.serve_seconds > 0:
        out["serving"] = serving_bench(torch, V, I, scene, args.serve_seconds)

    # ------------------------------------------------------------ CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(verts, tris, trace[warm:], I, fps)

    del img, lp
    result = {
        "metric": "frames/s + p99 frame ms, binocular 7680x4320 VaFR vs full-res ray cast, 1 GPU",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(1e3 * wall / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "binocular VaFR frame: 2 x (LP shading of 1,063,314 texels with primary + shadow ray "
                        "against 4,521,984 triangles, then inverse map to 7680x4320), 100x100 deg FOV, seeded "
                        "gaze trace",
            "display": [W, H], "eyes": 2, "triangles": int(tris.shape[0]), "lp_texels_per_eye": int(L.n_texels),
            "scene": SCENE,
        },
        "path": path,
        "batch_shape": tuned,
        "per_view_fps": round(fps_plain, 3),
        "per_view_p99_frame_ms": round(percentile(frame_ms_plain, 99), 4),
        "batched_fps": round(fps_batch, 3),
        "batched_p99_frame_ms": round(percentile(frame_ms_batch, 99), 4),
        "p50_frame_ms": round(percentile(frame_ms, 50), 4),
        "p99_frame_ms": round(percentile(frame_ms, 99), 4),
        "per_view_trace_ms_per_eye": round(float(np.mean(trace_ms)), 4),
        "per_view_reconstruct_ms_per_eye": round(float(np.mean(recon_ms)), 4),
        "batched_stage_ms": {"upload": round(b_upload_ms, 4), "trace": round(b_trace_ms, 4),
                             "reconstruct": round(b_recon_ms, 4), "frames": b_frames},
        "grays_per_s": round(rays_per_s / 1e9, 3),
        "display_gpix_per_s": round(2 * W * H * fps / 1e9, 3),
        "work_per_ray": {"node_visits": round(n_nodes / (n_prim + n_shadow), 2),
                         "triangle_tests": round(n_tri / (n_prim + n_shadow), 2),
                         "shadow_fraction": round(n_shadow / max(n_prim, 1), 3)},
        "roofline": {"kernel": k_trace, "bound": "alu", "achieved": round(achieved_gops, 1),
                     "peak": round(VALU_PEAK_GOPS, 1), "unit": "Gop/s",
                     "frac": round(achieved_gops / VALU_PEAK_GOPS, 4), "traffic": load_traffic(k_trace),
                     "launch_ms": round(trace_s * 1e3, 4), "ops_per_launch": int(ops_per_launch),
                     "ops_per_unit": {"node_visit": OPS_NODE, "triangle_test": OPS_TRI, "ray": OPS_RAY},
                     "frac_incl_node_format_decode": round(ops_fmt_per_launch / trace_s / 1e9 / VALU_PEAK_GOPS, 4),
                     "node_format_decode_ops_per_visit": OPS_NODE_FORMAT,
                     "counters": load_counters(k_trace)},
        "roofline_reconstruct": {"kernel": k_recon, "bound": "hbm", "achieved": round(recon_gbs, 1),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(recon_gbs / HBM_PEAK_GBS, 4),
                                 "traffic": load_traffic(k_recon), "launch_ms": round(recon_s * 1e3, 4),
                                 "bytes_per_launch": int(recon_bytes), "counters": load_counters(k_recon)},
        "cpu_baseline": cpu,
    }
    result.update(out)
    print(json.dumps(result), flush=True)


def pipelined_frames(torch, V, scene, cams, sh, L, gazes, warm, steps, shape):
    """Binocular 8K frames with two in flight: frame f runs as one batched
    frame on stream f mod 2 (the headline's autotuned launch shape), into its
    own LP buffers and display images, so the GPU overlaps one frame's
    reconstruction (HBM-bound) with the next frame's traversal (VALU-bound).
    Reports frames/s over the whole run and each frame's own duration (its
    events on its stream)."""
    lp = [[torch.empty((L.n_texels, 4), device="cuda") for _ in range(2)] for _ in range(2)]
    img = [[torch.empty((H * W, 4), device="cuda") for _ in range(2)] for _ in range(2)]
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    batches = [V.Batch(2, trace_block=shape["trace_block"], recon_rows=shape["recon_rows"], use_graph=True)
               for _ in range(2)]

    def frame(f, k, ev=None):
        if ev is not None:
            ev[0].record(streams[k])
        batches[k].run([V.view(V.VAFR_VIEW_VAFR, scene, cams[e], gazes[f], sh, layout=L, lp_rgba=lp[k][e],
                               img_rgba=img[k][e]) for e in range(2)], streams[k])
        if ev is not None:
            ev[1].record(streams[k])

    for f in range(warm):
        frame(f, f % 2)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for f in range(steps):
        frame(warm + f, f % 2, ev[f])
    torch.cuda.synchronize()
    fps = steps / (time.perf_counter() - t0)
    ms = [a.elapsed_time(b) for a, b in ev]
    for b in batches:
        b.close()
    log(f"pipelined (two frames in flight): {fps:.1f} frames/s, frame p50 {percentile(ms, 50):.3f} ms "
        f"p99 {percentile(ms, 99):.3f} ms")
    return {"frames": steps, "fps": round(fps, 2), "p50_frame_ms": round(percentile(ms, 50), 4),
            "p99_frame_ms": round(percentile(ms, 99), 4)}


def batch16(torch, V, I, scene, sh, steps):
    """16 views of display sizes drawn from 720p..8K with independent gaze
    on the shared 4.5M-triangle scene: one batched frame (one traversal + one
    reconstruction launch, graph replay, autotuned) against 16 separate
    shade + reconstruct call pairs."""
    sizes, gazes = I.batch_views(16, seed=4)
    cam = V.camera(I.terrain_camera())
    views = []
    for (W_, H_), g in zip(sizes, gazes):
        Lv = V.Layout.vafr(V.display(W_, H_, I.FOV))
        views.append((Lv, V.gaze(*g), torch.empty((Lv.n_texels, 4), device="cuda"),
                      torch.empty((W_ * H_, 4), device="cuda")))
    stream = torch.cuda.current_stream()
    desc = [V.view(V.VAFR_VIEW_VAFR, scene, cam, g, sh, layout=Lv, lp_rgba=lpv, img_rgba=imv)
            for Lv, g, lpv, imv in views]
    b = V.Batch(16)
    shape = b.autotune(desc, reps=3, stream=stream)

    def plain():
        for Lv, g, lpv, imv in views:
            V.vafr_shade_lp(scene, cam, g, sh, Lv, lpv, None, stream)
            V.vafr_reconstruct(Lv, g, lpv, imv, stream)

    res = {}
    for name, fn in (("plain", plain), ("batched", lambda: b.run(desc, stream))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        res[name] = steps / (time.perf_counter() - t0)
    pixels = sum(w * h for w, h in sizes)
    log(f"16 views ({pixels / 1e6:.1f} Mpix): batched {res['batched']:.1f} frames/s ({shape}), "
        f"16 plain call pairs {res['plain']:.1f} frames/s")
    b.close()
    return {"views": 16, "display_mpix": round(pixels / 1e6, 2), "batched_fps": round(res["batched"], 3),
            "plain_fps": round(res["plain"], 3), "speedup": round(res["batched"] / res["plain"], 3), "shape": shape}


def fxaa_bench(torch, V, scene, cams, sh, L, gazes, steps):
    """LP anti-aliasing (Sec. 3.4) on the binocular 8K frame: kernel time per
    eye, and per-view frames shade -> anti-alias -> inverse map."""
    stream = torch.cuda.current_stream()
    lp = [torch.empty((L.n_texels, 4), device="cuda") for _ in range(2)]
    aa = [torch.empty((L.n_texels, 4), device="cuda") for _ in range(2)]
    img = [torch.empty((H * W, 4), device="cuda") for _ in range(2)]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]

    def frame(f, timed=None):
        g = gazes[f % len(gazes)]
        for e in range(2):
            V.vafr_shade_lp(scene, cams[e], g, sh, L, lp[e], None, stream)
            if timed is not None and e == 0:
                timed[0].record(stream)
            V.vafr_fxaa_lp(L, lp[e], aa[e], stream)
            if timed is not None and e == 0:
                timed[1].record(stream)
            V.vafr_reconstruct(L, g, aa[e], img[e], stream)

    frame(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(steps):
        frame(f, ev[f])
    torch.cuda.synchronize()
    fps = steps / (time.perf_counter() - t0)
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    gbs = 2 * L.n_texels * 16 / (ms / 1e3) / 1e9
    log(f"LP anti-aliasing: {ms * 1e3:.1f} us per eye ({gbs:.0f} GB/s of LP read + write); per-view frames with it "
        f"{fps:.1f} frames/s")
    return {"us_per_eye": round(ms * 1e3, 2), "lp_gbs": round(gbs, 1), "per_view_fps_with_fxaa": round(fps, 2)}


def rep_bench(torch, V, scene, cams, sh, L, gazes, steps):
    """Binocular reprojection (Sec. 5.1): per-view frames whose right eye is
    warped from the left LP buffer (VaFR_Rep) against frames that shade both
    eyes (VaFR_Dup), same scene, cameras and gaze trace; the share of right
    texels the warp covered, and how far the warped right buffer is from
    the ray-cast one."""
    stream = torch.cuda.current_stream()
    lp = [torch.empty((L.n_texels, 4), device="cuda") for _ in range(2)]
    img = [torch.empty((H * W, 4), device="cuda") for _ in range(2)]
    ws = torch.empty(V.rep_workspace_bytes(L), device="cuda", dtype=torch.uint8)
    keys = ws[L.n_texels * 16:L.n_texels * 24].view(torch.int64)

    def rep(f):
        g = gazes[f % len(gazes)]
        V.vafr_shade_lp_rep(scene, cams[0], cams[1], g, sh, L, lp[0], lp[1], ws, None, None, stream)
        for e in range(2):
            V.vafr_reconstruct(L, g, lp[e], img[e], stream)

    side = torch.cuda.Stream()

    def rep2(f):
        # the right eye's ray-cast texels on a second stream, overlapping
        # the left eye's inverse map
        g = gazes[f % len(gazes)]
        V.vafr_shade_lp_rep(scene, cams[0], cams[1], g, sh, L, lp[0], lp[1], ws, None, None, stream, side)
        V.vafr_reconstruct(L, g, lp[0], img[0], stream)
        V.vafr_reconstruct(L, g, lp[1], img[1], side)
        stream.wait_stream(side)

    def dup(f):
        g = gazes[f % len(gazes)]
        for e in range(2):
            V.vafr_shade_lp(scene, cams[e], g, sh, L, lp[e], None, stream)
            V.vafr_reconstruct(L, g, lp[e], img[e], stream)

    res = {}
    for name, fn in (("dup", dup), ("rep", rep), ("rep2", rep2)):
        fn(0)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
        t0 = time.perf_counter()
        for f in range(steps):
            ev[f][0].record(stream)
            fn(f)
            ev[f][1].record(stream)
        torch.cuda.synchronize()
        fps = steps / (time.perf_counter() - t0)
        res[name] = (fps, float(np.mean([a.elapsed_time(b) for a, b in ev])))
    frac, dev = [], []
    for f in range(min(steps, 8)):
        dup(f)
        ref = lp[1].clone()
        rep(f)
        torch.cuda.synchronize()
        frac.append(float((keys != -1).float().mean()))
        dev.append(float((lp[1] - ref)[:, :3].abs().mean()))
    log(f"reprojection: Rep {res['rep'][0]:.1f} frames/s ({res['rep'][1]:.3f} ms), with the ray-cast texels on a "
        f"second stream {res['rep2'][0]:.1f} frames/s ({res['rep2'][1]:.3f} ms), Dup {res['dup'][0]:.1f} frames/s "
        f"({res['dup'][1]:.3f} ms); right texels warped {np.mean(frac):.3f}, mean |Rep - Dup| per channel "
        f"{np.mean(dev):.4f}")
    return {"rep_fps": round(res["rep"][0], 2), "rep_frame_ms": round(res["rep"][1], 3),
            "rep_two_stream_fps": round(res["rep2"][0], 2), "rep_two_stream_frame_ms": round(res["rep2"][1], 3),
            "dup_fps": round(res["dup"][0], 2), "dup_frame_ms": round(res["dup"][1], 3),
            "right_warped_frac": round(float(np.mean(frac)), 4),
            "right_mean_abs_diff_vs_dup": round(float(np.mean(dev)), 5), "per_view_path": True}


# Tangential-to-radial shading-rate ratio used to measure Eq. (19): 1 at the
# fovea, falling linearly to 1/2 at 30 deg (the sensitivity ratio the paper
# quotes there) and 1/2 beyond.
ANISO_EXAMPLE = ((0.0, 30.0), (1.0, 0.5))


def resolution_sweep(torch, V, I, scene, sh, cams, steps, full_steps, shape):
    """Binocular frames at the display sizes of Table 1 (2K, 4K, 6K, 8K and
    retinal 11520 x 6480 per eye): batched VaFR (same LP buffer at every
    size; the headline's autotuned launch shape) against
    the full-resolution ray cast (one primary + shadow ray per pixel).  Each
    size uses the seeded gaze trace scaled to its display."""
    sizes = [(2560, 1440), (3840, 2160), (5760, 3240), (7680, 4320), (11520, 6480)]
    stream = torch.cuda.current_stream()
    res = {}
    for Wd, Hd in sizes:
        disp = V.display(Wd, Hd, I.FOV)
        Ld = V.Layout.vafr(disp)
        tr = I.gaze_trace(steps + 10, Wd, Hd, seed=30)
        gz = [V.gaze(float(x), float(y)) for x, y in tr]
        lp = [torch.empty((Ld.n_texels, 4), device="cuda") for _ in range(2)]
        img = [torch.empty((Hd * Wd, 4), device="cuda") for _ in range(2)]
        b = V.Batch(2, trace_block=shape["trace_block"], recon_rows=shape["recon_rows"], use_graph=True)

        def frame(f):
            b.run([V.view(V.VAFR_VIEW_VAFR, scene, cams[e], gz[f], sh, layout=Ld, lp_rgba=lp[e], img_rgba=img[e])
                   for e in range(2)], stream)

        for f in range(5):
            frame(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(steps):
            frame(5 + f % (len(gz) - 5))
        torch.cuda.synchronize()
        vafr_fps = steps / (time.perf_counter() - t0)
        b.close()
        for e in range(2):
            V.full_shade(scene, cams[e], disp, sh, img[e], None, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(full_steps):
            for e in range(2):
                V.full_shade(scene, cams[e], disp, sh, img[e], None, stream)
        torch.cuda.synchronize()
        full_fps = full_steps / (time.perf_counter() - t0)
        key = f"{Wd}x{Hd}"
        res[key] = {"vafr_fps": round(vafr_fps, 2), "fullres_fps": round(full_fps, 3),
                    "speedup_vs_fullres": round(vafr_fps / full_fps, 2), "lp_texels_per_eye": Ld.n_texels,
                    "fullres_rays_per_eye": Wd * Hd}
        log(f"resolution {key}: VaFR {vafr_fps:.1f} frames/s, full resolution {full_fps:.2f} frames/s "
            f"({vafr_fps / full_fps:.1f}x)")
        del lp, img
    return res


def layout_variants(torch, V, I, scene, sh, cams, gazes, warm, steps, shape):
    """Binocular 8K batched frames for the paper's layout and its variants:
    device-adapted curves held at 9 and 18 cpd (Sec. 3.3) and an
    anisotropic tangential rate (Eq. (19)).  Same scene, cameras, gaze trace,
    launch shape (the headline's autotuned one) and warm-up as the headline
    batched frames."""
    variants = {"standard": V.Layout.vafr(V.display(W, H, I.FOV))}
    for cap in (9.0, 18.0):
        e, c = V.acuity_capped(cap)
        variants[f"cap{cap:g}cpd"] = V.Layout.vafr(V.display(W, H, I.FOV), e, c, 60.0)
    variants["anisotropic"] = V.Layout.vafr(V.display(W, H, I.FOV), aniso=ANISO_EXAMPLE)
    img = [torch.empty((H * W, 4), device="cuda") for _ in range(2)]
    stream = torch.cuda.current_stream()
    res = {}
    for name, Lv in variants.items():
        lp = [torch.empty((Lv.n_texels, 4), device="cuda") for _ in range(2)]
        b = V.Batch(2, trace_block=shape["trace_block"], recon_rows=shape["recon_rows"], use_graph=True)

        def frame(f):
            g = gazes[f % len(gazes)]
            b.run([V.view(V.VAFR_VIEW_VAFR, scene, cams[e], g, sh, layout=Lv, lp_rgba=lp[e], img_rgba=img[e])
                   for e in range(2)], stream)

        for f in range(warm):
            frame(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(steps):
            frame(warm + f)
        torch.cuda.synchronize()
        fps = steps / (time.perf_counter() - t0)
        res[name] = {"columns": Lv.n_cols, "texels_per_eye": Lv.n_texels, "fps": round(fps, 2), "frames": steps}
        log(f"layout {name}: {Lv.n_cols} columns, {Lv.n_texels} texels per eye, {fps:.1f} frames/s")
        b.close()
        del lp
    return res


def serving_bench(torch, V, I, scene4m, seconds):
    """8 headsets at 90 Hz with Poisson arrivals, binocular displays 2K x 3,
    4K x 3, 8K x 2, even headsets on the 1.13M-triangle scene and odd ones on
    the 4.52M-triangle scene, path-traced LP shading (1 sample, 2 bounces).
    The continuous-batching server is compared with the same server limited
    to one request per launch and one launch at a time (plain per-view
    launches).  Both run with an 11.1 ms frame budget (one 90 Hz refresh)
    and latest-frame replacement: requests the device cannot finish within
    the budget are dropped before launch and counted, as a VR compositor
    would re-show the previous frame.  Latency = request submit -> both
    eyes' images ready."""
    from paper_2503_23410_amd import serving
    scene1m = V.Scene(*I.make_scene("terrain1m"))
    sizes = [(2560, 1440)] * 3 + [(3840, 2160)] * 3 + [(7680, 4320)] * 2
    layouts = {sz: V.Layout.vafr(V.display(sz[0], sz[1], I.FOV)) for sz in set(sizes)}
    sh = V.shading(mode=V.VAFR_SHADE_PATH, bounces=2, seed=2025)
    cl, cr = (V.camera(c) for c in I.binocular_cameras())
    arrivals = serving.arrival_times(8, 90.0, seconds, seed_base=5)
    gazes = [I.gaze_trace(int(seconds * 200) + 50, w, h, seed=40 + k) for k, (w, h) in enumerate(sizes)]
    res = {"headsets": 8, "rate_hz": 90, "seconds": seconds, "requests": len(arrivals),
           "displays": "2560x1440 x3, 3840x2160 x3, 7680x4320 x2 (binocular)", "shading": "path, 1 spp, 2 bounces"}
    res["frame_budget_ms"] = FRAME_BUDGET_MS
    for name, kw in (("batched", dict(max_views_per_launch=16, max_inflight=2, n_streams=1)),
                     ("plain", dict(max_views_per_launch=2, max_inflight=1, n_streams=1))):
        srv = V.Server(max_queue=256, hbm_budget_bytes=64 << 30, frame_budget_ms=FRAME_BUDGET_MS, latest_only=True,
                       watchdog_ms=2000.0, **kw)
        for k, sz in enumerate(sizes):
            srv.add_headset(scene1m if k % 2 == 0 else scene4m, layouts[sz], cl, cr, sh)
        # warm-up: one request per headset (buffers, graphs)
        for k in range(8):
            srv.submit(k, 10 ** 6 + k, V.gaze(sizes[k][0] / 2, sizes[k][1] / 2))
        srv.wait_idle(120000)
        for r in srv.poll():
            if r["status"] == 0:
                srv.release(r["slot"])
        st0 = srv.stats()
        recs, refused, wall = serving.run(srv, V, gazes, arrivals)
        st = srv.stats()
        lat = serving.latency_stats(recs)
        launches = st["launches"] - st0["launches"]
        entry = {"frames_per_s": round(lat["completed"] / wall, 2),
                 "completion_rate": round(lat["completed"] / max(len(arrivals), 1), 4),
                 "p50_ms": round(lat["p50_ms"], 3),
                 "p99_ms": round(lat["p99_ms"], 3), "max_ms": round(lat["max_ms"], 3),
                 "mean_queue_ms": round(lat["mean_queue_ms"], 3), "completed": lat["completed"],
                 "refused": refused, "late": st["late"] - st0["late"],
                 "superseded": st["superseded"] - st0["superseded"], "stalled": st["stalled"] - st0["stalled"],
                 "deferred": st["deferred"] - st0["deferred"], "launches": launches,
                 "requests_per_launch": round(lat["completed"] / max(launches, 1), 2)}
        log(f"serving ({name}): {entry}")
        res[name] = entry
        srv.close()
    return res


def cpu_baseline(verts, tris, gazes, I, gpu_fps=None):
    """The oracle on the host cores, as it stands, in the same run: the
    headline workload on all host threads and on one thread, each stage
    timed on its own.  Bounded samples keep the whole leg to about 10-20 s
    of host time:
      - layout (FP64 tables) and the oracle's BVH build: timed once;
      - VaFR, all threads: 2 whole binocular frames (every LP texel of both
        eyes shaded with primary + shadow rays, every display pixel
        reconstructed in bands of rows);
      - VaFR, one thread: 1 binocular frame on a seeded 1/16 of the LP
        texels and 1/64 of the display pixels, extrapolated;
      - full resolution (GT): a seeded 1/64 of each eye's pixels (all
        threads; 1/256 on one thread), extrapolated;
      - LMFR(1.8): a seeded 1/64 of the LP texels and of the display pixels
        (1/256 on one thread), extrapolated."""
    import oracle as O
    thr = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    rng = np.random.default_rng(77)
    t0 = time.perf_counter()
    lay = O.Layout()
    t_layout = time.perf_counter() - t0
    t0 = time.perf_counter()
    osc = O.Scene(verts, tris)
    t_bvh = time.perf_counter() - t0
    p = O.film_pitch(W, H, *I.FOV)
    cams = I.binocular_cameras()
    sh = O.shading_params()
    lw, lh = O.lmfr_dims(W, H, 1.8)
    band = H // 8

    def subset(n, frac):
        return np.sort(rng.choice(n, max(1, int(n * frac)), replace=False))

    def run(threads, n_frames, tex_frac, pix_frac, gt_frac, lm_frac):
        O.set_threads(threads)
        used = O.get_threads()
        t_shade = t_recon = t_full = t_lmfr = 0.0
        for f in range(n_frames):
            gaze = (float(gazes[f][0]), float(gazes[f][1]))
            G = O.gaze_film(W, H, p, *gaze)
            for cam in cams:
                idx = np.arange(lay.n_texels) if tex_frac == 1 else subset(lay.n_texels, tex_frac)
                a = time.perf_counter()
                lp, _, _ = O.shade_vafr_texels(osc, lay, idx, W, H, I.FOV, gaze, cam, sh)
                t_shade += (time.perf_counter() - a) / tex_frac
                full_lp = lp if tex_frac == 1 else np.zeros((lay.n_texels, 4), np.float32)
                if pix_frac == 1:
                    for y0 in range(0, H, band):
                        pix = np.arange(y0 * W, min(H, y0 + band) * W, dtype=np.int64)
                        a = time.perf_counter()
                        O.vafr_reconstruct(lay, full_lp, W, H, p, G, pix)
                        t_recon += time.perf_counter() - a
                else:
                    pix = subset(W * H, pix_frac)
                    a = time.perf_counter()
                    O.vafr_reconstruct(lay, full_lp, W, H, p, G, pix)
                    t_recon += (time.perf_counter() - a) / pix_frac
            # comparisons on the first frame's gaze, both eyes
            if f == 0:
                for cam in cams:
                    pix = subset(W * H, gt_frac)
                    a = time.perf_counter()
                    O.shade_full_pixels(osc, pix, W, H, I.FOV, cam, sh)
                    t_full += (time.perf_counter() - a) / gt_frac
                    idx = subset(lw * lh, lm_frac)
                    a = time.perf_counter()
                    O.shade_lmfr_texels(osc, idx, W, H, I.FOV, gaze, lw, lh, 4.0, cam, sh)
                    b = time.perf_counter()
                    O.lmfr_reconstruct(W, H, gaze[0], gaze[1], lw, lh, 4.0, np.zeros((lw * lh, 4), np.float32),
                                       subset(W * H, lm_frac))
                    t_lmfr += (b - a + time.perf_counter() - b) / lm_frac
        per = (t_shade + t_recon) / n_frames
        return {"fps": n_frames / (t_shade + t_recon), "threads": used,
                "shade_s_per_frame": round(t_shade / n_frames, 4), "reconstruct_s_per_frame": round(t_recon / n_frames, 4),
                "frame_s": round(per, 4), "fullres_fps": round(1.0 / t_full, 6), "lmfr_fps": round(1.0 / t_lmfr, 6)}

    many = run(thr, 2, 1, 1, 1 / 64, 1 / 64)
    one = run(1, 1, 1 / 16, 1 / 64, 1 / 256, 1 / 256)
    log(f"oracle: layout {t_layout:.3f}s, BVH build {t_bvh:.2f}s (once); {many['threads']} threads: "
        f"{many['fps']:.4f} binocular VaFR frames/s (shade {many['shade_s_per_frame']:.2f}s + reconstruct "
        f"{many['reconstruct_s_per_frame']:.2f}s per frame), full resolution {many['fullres_fps']:.5f} frames/s, "
        f"LMFR(1.8) {many['lmfr_fps']:.5f} frames/s; 1 thread: {one['fps']:.5f} VaFR frames/s, full resolution "
        f"{one['fullres_fps']:.6f}, LMFR {one['lmfr_fps']:.6f}")
    res = {"value": round(many["fps"], 5), "unit": "frames/s", "cores": many["threads"], "kind": "oracle",
           "sample": f"VaFR binocular 7680x4320 frames on {many['threads']} threads: 2 whole frames (2 x "
                     f"{lay.n_texels} LP texels with primary + shadow rays, 2 x {W}x{H} pixels reconstructed), "
                     f"gazes from the same trace; the oracle's layout and BVH build are timed apart "
                     f"(stages_s); full resolution and LMFR(1.8) on a seeded 1/64 of their rays / texels and "
                     f"pixels, extrapolated",
           "stages_s": {"layout": round(t_layout, 4), "bvh_build": round(t_bvh, 3),
                        "shade_per_frame": many["shade_s_per_frame"],
                        "reconstruct_per_frame": many["reconstruct_s_per_frame"]},
           "fullres_fps": many["fullres_fps"], "lmfr_fps": many["lmfr_fps"],
           "single_thread": {"value": round(one["fps"], 6), "unit": "frames/s", "cores": one["threads"],
                             "sample": "1 binocular frame on a seeded 1/16 of the LP texels and 1/64 of the "
                                       "display pixels, extrapolated; full resolution and LMFR(1.8) on a "
                                       "seeded 1/256, extrapolated",
                             "shade_s_per_frame": one["shade_s_per_frame"],
                             "reconstruct_s_per_frame": one["reconstruct_s_per_frame"],
                             "fullres_fps": one["fullres_fps"], "lmfr_fps": one["lmfr_fps"]}}
    if gpu_fps:
        res["gpu_over_oracle"] = round(gpu_fps / many["fps"], 1)
    return res


# ---------------------------------------------------------------- profiles
# `python bench.py --profile-summary DIR` turns rocprofv3 output written
# under DIR by the commands listed in PROFILE_COMMANDS (run from the
# repository root with TMPDIR=/tmp, each under its own timeout) into the
# summaries under profiles/ and the per-kernel traffic / counter files that
# the benchmark reports while the kernel sources are unchanged.
_HEAD = ("python3 bench.py --steps 200 --warmup 20 --no-cpu-baseline --no-compare --serve-seconds 0 "
         "--no-pipelined")
_SHORT = ("python3 bench.py --steps 10 --warmup 2 --no-cpu-baseline --no-compare --serve-seconds 0 "
          "--no-pipelined")
_SERVE = "python3 bench.py --steps 5 --warmup 2 --no-cpu-baseline --no-compare --no-pipelined --serve-seconds 3"
_COPY = ("python3 -c \"import torch; a=torch.ones(1<<28, device='cuda'); b=torch.empty_like(a); "
         "torch.cuda.synchronize(); [b.copy_(a) for _ in range(4)]; torch.cuda.synchronize(); print('copy done')\"")
_SQ1 = "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_SALU SQ_INSTS_LDS GRBM_GUI_ACTIVE"
_SQ2 = "SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_WAIT_ANY TCC_HIT_sum TCC_MISS_sum"
PROFILE_COMMANDS = {
    "kt": f"rocprofv3 --kernel-trace --stats --output-format csv -d DIR/kt -o run -- {_HEAD} > DIR/kt.json",
    "kts": f"rocprofv3 --kernel-trace --stats --output-format csv -d DIR/kts -o run -- {_SERVE} > DIR/kts.json",
    "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/fetch -o run -- {_SHORT}",
    "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/write -o run -- {_SHORT}",
    "copy_fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/copy_fetch -o run -- {_COPY}",
    "copy_write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/copy_write -o run -- {_COPY}",
    "sq1": f"rocprofv3 --pmc {_SQ1} --output-format csv -d DIR/sq1 -o run -- {_SHORT}",
    "sq2": f"rocprofv3 --pmc {_SQ2} --output-format csv -d DIR/sq2 -o run -- {_SHORT}",
    "sq1s": f"rocprofv3 --pmc {_SQ1} --output-format csv -d DIR/sq1s -o run -- {_SERVE}",
    "sq2s": f"rocprofv3 --pmc {_SQ2} --output-format csv -d DIR/sq2s -o run -- {_SERVE}",
}


def _short_kernel(name):
    """Kernel name without namespace, return type and parameter list."""
    for pre in ("vafr::(anonymous namespace)::", "void "):
        name = name.replace(pre, "")
    name = name.strip()
    if name.endswith(")"):
        depth = 0
        for i in range(len(name) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(name[i], 0)
            if depth == 0:
                name = name[:i]
                break
    return name.strip()


def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows += list(csv.DictReader(f))
    return rows


def _col(row, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(names)


def _kernel_stats(d):
    """Per kernel: calls, mean / min / max duration in microseconds, grid."""
    out = {}
    for r in _csv_rows(d, "kernel_trace.csv"):
        k = _short_kernel(_col(r, "Kernel_Name"))
        dur = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        grid = int(_col(r, "Grid_Size_X", "Grid_Size"))
        e = out.setdefault(k, {"calls": 0, "sum": 0.0, "min": 1e30, "max": 0.0, "grid": grid})
        e["calls"] += 1
        e["sum"] += dur
        e["min"] = min(e["min"], dur)
        e["max"] = max(e["max"], dur)
    for e in out.values():
        e["avg"] = e["sum"] / e["calls"]
    return out


def _counters(d):
    """Per (kernel, grid): mean of each counter over the dispatches."""
    acc = {}
    for r in _csv_rows(d, "counter_collection.csv"):
        k = (_short_kernel(_col(r, "Kernel_Name")), int(_col(r, "Grid_Size")))
        c = _col(r, "Counter_Name")
        disp = _col(r, "Dispatch_Id", "Correlation_Id")
        e = acc.setdefault(k, {}).setdefault(c, {})
        e[disp] = e.get(disp, 0.0) + float(_col(r, "Counter_Value"))
    return {k: {c: sum(v.values()) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def _bench_json(path):
    try:
        with open(path) as f:
            lines = [ln for ln in f.read().splitlines() if ln.startswith("{")]
        return json.loads(lines[-1]) if lines else None
    except OSError:
        return None


def profile_summary(d):
    prof = os.path.join(ROOT, "profiles")
    h = kernel_source_hash()
    cmd = lambda k: PROFILE_COMMANDS[k].replace("DIR", d)
    lines = []
    # ---- kernel trace of the headline frames (and the roofline from it)
    kt = _kernel_stats(os.path.join(d, "kt"))
    bj = _bench_json(os.path.join(d, "kt.json"))
    L = ["Kernel trace, binocular 7680x4320 VaFR on the 4,521,984-triangle terrain: per-view frames, then the",
         "autotuner and the batched frames (one traversal + one reconstruction launch per frame, graph replay);",
         "the two-frames-in-flight, comparison, serving and oracle legs are off, so no launch overlaps another.",
         "", "Command (repository root, TMPDIR=/tmp):", "  " + cmd("kt"), "",
         f"{'kernel':<52}{'grid':>10}{'calls':>7}{'avg us':>10}{'min us':>9}{'max us':>9}"]
    for k, e in sorted(kt.items(), key=lambda kv: -kv[1]["sum"]):
        L.append(f"{k:<52}{e['grid']:>10}{e['calls']:>7}{e['avg']:>10.2f}{e['min']:>9.2f}{e['max']:>9.2f}")
    if bj:
        rt, rr = bj["roofline"], bj["roofline_reconstruct"]
        shape = bj.get("batch_shape", {})
        kt_name = f"k_trace_batch<{shape.get('trace_block', 128)}, 24, false, false, true>"
        kr_name = f"k_recon_batch<{shape.get('recon_rows', 8)}>"
        L += ["", f"Roofline from these averages (work per launch from the same run's JSON line, {kt_name} and "
                  f"{kr_name}):"]
        if kt_name in kt:
            a = kt[kt_name]["avg"] / 1e6
            fr = rt["ops_per_launch"] / a / 1e9 / VALU_PEAK_GOPS
            fr_fmt = rt["frac_incl_node_format_decode"] * rt["launch_ms"] / 1e3 / a
            L.append(f"  traversal: {rt['ops_per_launch']:,} algorithmic ops / {a * 1e6:.2f} us = "
                     f"{rt['ops_per_launch'] / a / 1e9:.0f} Gop/s = {fr:.3f} of {VALU_PEAK_GOPS:.0f} Gop/s "
                     f"({fr_fmt:.3f} counting the node-format decode); the bench line's event time "
                     f"{rt['launch_ms'] * 1e3:.2f} us gives {rt['frac']:.3f}")
        if kr_name in kt:
            a = kt[kr_name]["avg"] / 1e6
            gbs = rr["bytes_per_launch"] / a / 1e9
            L.append(f"  reconstruction: {rr['bytes_per_launch'] / 1e6:.1f} MB / {a * 1e6:.2f} us = {gbs:.0f} GB/s "
                     f"= {gbs / HBM_PEAK_GBS:.3f} of {HBM_PEAK_GBS:.0f} GB/s; the bench line's event time "
                     f"{rr['launch_ms'] * 1e3:.2f} us gives {rr['frac']:.3f}")
    _write(os.path.join(prof, "binocular8k_kernel_trace.txt"), L)
    # ---- serving kernels
    kts = _kernel_stats(os.path.join(d, "kts"))
    L = ["Kernel trace of the served workload: 8 headsets at 90 Hz (binocular 2560x1440 x3, 3840x2160 x3,",
         "7680x4320 x2; 1.13M / 4.52M-triangle terrains), path-traced LP shading (1 sample, 2 bounces), 11.1 ms",
         "frame budget, 3 s per server configuration (continuous batching, then one request per launch), after",
         "a short headline run (5 frames).  Path-mode kernels: k_trace_batch<..., true, false> (bounces 0-1,",
         "live paths queued) and k_trace_queue_batch (the queued second bounce).", "",
         "Command (repository root, TMPDIR=/tmp):", "  " + cmd("kts"), "",
         f"{'kernel':<52}{'grid':>10}{'calls':>7}{'avg us':>10}{'min us':>9}{'max us':>9}{'total ms':>10}"]
    for k, e in sorted(kts.items(), key=lambda kv: -kv[1]["sum"]):
        L.append(f"{k:<52}{e['grid']:>10}{e['calls']:>7}{e['avg']:>10.2f}{e['min']:>9.2f}{e['max']:>9.2f}"
                 f"{e['sum'] / 1e3:>10.1f}")
    _write(os.path.join(prof, "serving_path_kernel_trace.txt"), L)
    # ---- HBM traffic
    fe, wr = _counters(os.path.join(d, "fetch")), _counters(os.path.join(d, "write"))
    cf, cw = _counters(os.path.join(d, "copy_fetch")), _counters(os.path.join(d, "copy_write"))
    copy_kib = (1 << 30) / 1024.0
    cfk = max((v.get("FETCH_SIZE", 0.0) for v in cf.values()), default=0.0)
    cwk = max((v.get("WRITE_SIZE", 0.0) for v in cw.values()), default=0.0)
    sf = copy_kib / cfk if cfk else 1.0
    sw = copy_kib / cwk if cwk else 1.0
    L = ["HBM traffic per launch from rocprofv3 PMC counters (one counter per run), binocular 7680x4320 VaFR.",
         "", "Commands (repository root, TMPDIR=/tmp, each under timeout -s KILL):"]
    L += ["  " + cmd(k) for k in ("fetch", "write", "copy_fetch", "copy_write")]
    L += ["", f"Calibration: a 1 GiB device copy reads FETCH_SIZE = {cfk:.0f} KiB and WRITE_SIZE = {cwk:.0f} KiB "
              f"per dispatch, so", f"FETCH_SIZE is scaled by {sf:.3f} and WRITE_SIZE by {sw:.3f}.", "",
          f"{'kernel':<52}{'grid':>10}{'FETCH KiB':>12}{'WRITE KiB':>12}{'HBM MB/launch':>15}"]
    traffic = {}
    for key in sorted(set(fe) & set(wr)):
        f_k, w_k = fe[key].get("FETCH_SIZE", 0.0), wr[key].get("WRITE_SIZE", 0.0)
        mb = (f_k * sf + w_k * sw) * 1024 / 1e6
        L.append(f"{key[0]:<52}{key[1]:>10}{f_k:>12.0f}{w_k:>12.0f}{mb:>15.1f}")
        for kind, pre in (("k_trace_batch", "k_trace_batch<"), ("k_recon_batch", "k_recon_batch<")):
            if key[0].startswith(pre) and bj:
                shape = bj.get("batch_shape", {})
                want = (f"k_trace_batch<{shape.get('trace_block', 128)}, 24, false, false, true>"
                        if kind == "k_trace_batch" else f"k_recon_batch<{shape.get('recon_rows', 8)}>")
                if key[0] == want:
                    traffic[kind] = {"source_hash": h, "bytes_per_launch": int(mb * 1e6),
                                     "calibration": {"fetch": round(sf, 4), "write": round(sw, 4)},
                                     "kernel": want, "source": "profiles/binocular8k_hbm_traffic.txt"}
    L += ["", "Algorithmic bytes: reconstruction of a binocular frame writes 2 x 33,177,600 x 16 B = 1061.7 MB and",
          "reads the two LP buffers once (2 x 1,063,314 x 16 B = 34.0 MB): 1095.7 MB.  Traversal writes the two LP",
          "buffers (34.0 MB) and reads the texel offsets and order (2 x 12.8 MB) besides the BVH and triangles",
          "(287 MB resident, mostly served from L2 and the Infinity Cache)."]
    _write(os.path.join(prof, "binocular8k_hbm_traffic.txt"), L)
    if traffic:
        with open(os.path.join(prof, "pmc_traffic.json"), "w") as f:
            json.dump(traffic, f, indent=1)
    # ---- SQ counters
    sq = {}
    L = ["Shader-sequencer and L2 counters (two passes per workload), binocular 7680x4320 VaFR and the served",
         "path-traced workload.", "", "Commands (repository root, TMPDIR=/tmp, each under timeout -s KILL):"]
    L += ["  " + cmd(k) for k in ("sq1", "sq2", "sq1s", "sq2s")]
    L.append("")
    seen = set()
    for a, b in (("sq1", "sq2"), ("sq1s", "sq2s")):
        c1, c2 = _counters(os.path.join(d, a)), _counters(os.path.join(d, b))
        for key in sorted(set(c1) & set(c2), key=lambda k: (k[0], k[1])):
            if not key[0].startswith(("k_trace", "k_recon")) or key[0].startswith("k_trace_plan"):
                continue
            # the serving run starts with a short headline run: list only its own kernels
            if a == "sq1s" and key[0] in seen:
                continue
            if a == "sq1":
                seen.add(key[0])
            x = {**c1[key], **c2[key]}
            cyc = x.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
            if cyc <= 0 or not x.get("SQ_WAVES"):
                continue
            valu = x.get("SQ_INSTS_VALU", 0.0)
            per_clk = valu / (1024.0 * cyc)
            lanes = x.get("SQ_THREAD_CYCLES_VALU", 0.0) / max(x.get("SQ_ACTIVE_INST_VALU", 1.0), 1.0) / 64.0
            resident = x.get("SQ_WAVE_CYCLES", 0.0) * 4.0 / (1024.0 * cyc)
            wait = x.get("SQ_WAIT_ANY", 0.0) / max(x.get("SQ_WAVE_CYCLES", 1.0), 1.0)
            hit = x.get("TCC_HIT_sum", 0.0) / max(x.get("TCC_HIT_sum", 0.0) + x.get("TCC_MISS_sum", 0.0), 1.0)
            L.append(f"{key[0]} (grid {key[1]}, {'served' if a == 'sq1s' else 'headline'}): GRBM_GUI_ACTIVE/8 = "
                     f"{cyc:.0f} cycles; VALU instructions {valu:.0f} ({valu / x['SQ_WAVES']:.0f} per wave), SALU "
                     f"{x.get('SQ_INSTS_SALU', 0):.0f}, VMEM {x.get('SQ_INSTS_VMEM_RD', 0):.0f}, LDS "
                     f"{x.get('SQ_INSTS_LDS', 0):.0f}; wave64 VALU instructions per SIMD per clock {per_clk:.3f}; "
                     f"active lanes per VALU instruction {lanes:.0%}; mean resident waves per SIMD {resident:.1f}; "
                     f"waves waiting {wait:.0%} of their cycles; L2 hit rate {hit:.0%}")
            L.append("")
            entry = {"source_hash": h, "grid": key[1], "valu_per_simd_clock": round(per_clk, 4),
                     "active_lane_frac": round(lanes, 4), "resident_waves_per_simd": round(resident, 2),
                     "wait_frac": round(wait, 4), "source": "profiles/sq_counters.txt"}
            if a == "sq1" and bj:
                shape = bj.get("batch_shape", {})
                if key[0] == f"k_trace_batch<{shape.get('trace_block', 128)}, 24, false, false, true>":
                    sq["k_trace_batch"] = {**entry, "kernel": key[0]}
                if key[0] == f"k_recon_batch<{shape.get('recon_rows', 8)}>":
                    sq["k_recon_batch"] = {**entry, "kernel": key[0]}
            sq.setdefault("by_kernel", {})[f"{key[0]} grid {key[1]}"] = entry
    L += ["Cycles are GRBM_GUI_ACTIVE summed over the 8 XCDs divided by 8 (it matches the kernel duration at",
          "2.4 GHz).  Active lanes = SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU / 64.  Resident waves =",
          "SQ_WAVE_CYCLES (quad-cycles) x 4 / (1024 SIMDs x cycles).  Waiting = SQ_WAIT_ANY / SQ_WAVE_CYCLES."]
    _write(os.path.join(prof, "sq_counters.txt"), L)
    if sq:
        with open(os.path.join(prof, "pmc_sq.json"), "w") as f:
            json.dump(sq, f, indent=1)
    print(f"profiles written from {d} (kernel source hash {h})")


def _write(path, lines):
    with open(path, "w") as f:
        f.write("\n".join(lines).rstrip() + "\n")


if __name__ == "__main__":
    main()
