"""The paths the benchmark times, compared directly with the oracle (not
with other HIP calls):

1. The batched binocular frame exactly as the benchmark launches it: two
   7680 x 4320 VaFR views on the 4,521,984-triangle terrain, Lambert + shadow
   ray, one traversal and one reconstruction launch per frame replayed from a
   hipGraph, launch shape chosen by the autotuner.  Frames after the
   autotuner's timing runs traverse in the longest-first order that
   k_trace_plan derives from the previous frame's block durations, so the
   two frames checked here (different gazes of the seeded trace) both run
   planned.
2. One served 8K path-traced request (1 sample, 2 bounces; bounces after
   the first run from the batch's compacted queue of live paths), submitted
   together with a 2K request of another headset so that both share a
   launch.

Acceptance (Sec. 6.1 pipeline; tolerances of the parity contract): hit ids
identical on unflagged rays, colours within 2e-3 on unflagged texels and
pixels, flagged rays at most 1e-4 of the LP texels; every LP texel of both
eyes, and at least 300,000 display pixels per eye plus the whole last row
and column.
"""
import sys

import numpy as np
import pytest

from paper_2503_23410_amd import inputs as I

pytestmark = pytest.mark.gpu

COLOR_TOL = 2e-3
FLAG_FRAC = 1e-4
W, H = 7680, 4320


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env(O):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_23410_amd import vafr as V
    V.load()
    O.set_threads(16)
    return torch, V


@pytest.fixture(scope="module")
def terrain4m(env, O):
    torch, V = env
    v, f = I.make_scene("terrain4m")
    return V.Scene(v, f), O.Scene(v, f)


def _check_lp(name, g_rgba, g_id, o_rgba, o_id, o_fl):
    unf = o_fl == 0
    n = len(o_fl)
    nflag = int((~unf).sum())
    diff = np.abs(g_rgba - o_rgba).max(axis=1)
    worst = float(diff[unf].max())
    mism = int(((g_id != o_id) & unf).sum()) if g_id is not None else -1
    log(f"{name}: texels={n} flagged={nflag} ({nflag / n:.2e}) id_mismatch_unflagged={mism} "
        f"max_colour_err={worst:.2e} hit_frac={(o_id >= 0).mean():.3f}")
    if g_id is not None:
        assert mism == 0, f"{name}: {mism} unflagged hit-id mismatches"
    assert nflag <= FLAG_FRAC * n, f"{name}: {nflag} flagged rays exceed 1e-4 of {n}"
    assert worst <= COLOR_TOL, f"{name}: colour error {worst}"


def _pixels(rng, n=300000):
    edge = np.concatenate([(H - 1) * W + np.arange(W), np.arange(H) * W + (W - 1)])
    return np.unique(np.concatenate([rng.integers(0, W * H, n), edge]))


def _check_image(torch, O, name, layout, img, o_lp, o_fl, gz, pix):
    p = O.film_pitch(W, H, *I.FOV)
    ref, pf = O.vafr_reconstruct(layout, o_lp, W, H, p, O.gaze_film(W, H, p, *gz), pix, o_fl)
    g = img[torch.from_numpy(pix).cuda()].cpu().numpy()
    err = np.abs(g - ref).max(axis=1)
    log(f"{name}: pixels={len(pix)} flagged_px={int(pf.sum())} max_err_unflagged={err[~pf].max():.2e}")
    assert err[~pf].max() <= COLOR_TOL


def test_batched_headline_frames_match_oracle(env, O, layout, terrain4m):
    torch, V = env
    g_sc, o_sc = terrain4m
    L = V.Layout.vafr(V.display(W, H, I.FOV))
    assert L.n_texels == layout.n_texels
    cams = I.binocular_cameras()
    vcams = [V.camera(c) for c in cams]
    sh = V.shading()
    trace = I.gaze_trace(60, W, H, seed=30)
    frames = (20, 37)
    gz = [(float(trace[f, 0]), float(trace[f, 1])) for f in frames]
    assert gz[0] != gz[1]
    n = L.n_texels
    lp = [[torch.full((n, 4), -1.0, device="cuda") for _ in range(2)] for _ in frames]
    hid = [torch.full((n,), -9, device="cuda", dtype=torch.int32) for _ in range(2)]
    img = [[torch.full((W * H, 4), -1.0, device="cuda") for _ in range(2)] for _ in frames]
    batch = V.Batch(2)

    def views(k, with_ids):
        return [V.view(V.VAFR_VIEW_VAFR, g_sc, vcams[e], V.gaze(*gz[k]), sh, layout=L, lp_rgba=lp[k][e],
                       hit_id=hid[e] if with_ids else None, img_rgba=img[k][e]) for e in range(2)]

    tuned = batch.autotune(views(0, False), reps=5)
    log(f"autotuned launch shape: {tuned}")
    assert tuned["use_graph"] == 1
    # frame 0 also writes hit ids; frame 1 is the benchmark's exact descriptor
    # (no hit-id buffer)
    batch.run(views(0, True))
    batch.run(views(1, False))
    torch.cuda.synchronize()
    rng = np.random.default_rng(33)
    for k in range(2):
        for e in range(2):
            o_rgba, o_id, o_fl = O.shade_vafr_texels(o_sc, layout, np.arange(n), W, H, I.FOV, gz[k], cams[e],
                                                     O.shading_params())
            g_id = hid[e].cpu().numpy() if k == 0 else None
            _check_lp(f"batched frame {frames[k]} eye {e} LP", lp[k][e].cpu().numpy(), g_id, o_rgba, o_id, o_fl)
            _check_image(torch, O, f"batched frame {frames[k]} eye {e} image", layout, img[k][e], o_rgba, o_fl,
                         gz[k], _pixels(rng))
    batch.close()


def test_served_8k_path_request_matches_oracle(env, O, layout, terrain4m):
    torch, V = env
    g_sc, o_sc = terrain4m
    L8 = V.Layout.vafr(V.display(W, H, I.FOV))
    L2 = V.Layout.vafr(V.display(2560, 1440, I.FOV))
    seed = 2025
    sh = V.shading(mode=V.VAFR_SHADE_PATH, bounces=2, seed=seed)
    cams = I.binocular_cameras()
    srv = V.Server(max_views_per_launch=16, max_inflight=2, n_streams=1, max_queue=64, hbm_budget_bytes=16 << 30)
    h2 = srv.add_headset(g_sc, L2, V.camera(cams[0]), V.camera(cams[1]), sh)
    h8 = srv.add_headset(g_sc, L8, V.camera(cams[0]), V.camera(cams[1]), sh)
    g8 = I.gaze_trace(40, W, H, seed=41)[23]
    g2 = I.gaze_trace(40, 2560, 1440, seed=42)[11]
    gz8, gz2 = (float(g8[0]), float(g8[1])), (float(g2[0]), float(g2[1]))
    f8, f2 = 77, 78
    assert srv.submit(h2, f2, V.gaze(*gz2)) and srv.submit(h8, f8, V.gaze(*gz8))
    srv.wait_idle(60000)
    res = {r["headset"]: r for r in srv.poll()}
    st = srv.stats()
    assert set(res) == {h2, h8} and all(r["status"] == 0 for r in res.values())
    log(f"served: {st['launches']} launch(es) for 2 requests")
    assert st["launches"] == 1, "the two requests should share one batched launch"
    n = layout.n_texels
    rng = np.random.default_rng(44)
    for h, Lh, gz, fr, (w, hh) in ((h8, L8, gz8, f8, (W, H)), (h2, L2, gz2, f2, (2560, 1440))):
        for e in range(2):
            lp = torch.empty((n, 4), device="cuda")
            V.copy_from_device(lp, res[h]["lp"][e])
            p = O.film_pitch(w, hh, *I.FOV)
            org, d = O.vafr_rays(layout, np.arange(n), O.gaze_film(w, hh, p, *gz), cams[e])
            o_rgba, o_id, o_fl = o_sc.shade_path(org, d, np.arange(n), O.shading_params(), seed, fr, 2 * h + e, 2)
            _check_lp(f"served {w}x{hh} path eye {e} LP", lp.cpu().numpy(), None, o_rgba, o_id, o_fl)
            if h == h8:
                img = torch.empty((W * H, 4), device="cuda")
                V.copy_from_device(img, res[h]["img"][e])
                _check_image(torch, O, f"served 8K path eye {e} image", layout, img, o_rgba, o_fl, gz, _pixels(rng))
                del img
        srv.release(res[h]["slot"])
    srv.close()
