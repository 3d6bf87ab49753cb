"""Serving loop on the GPU: a served frame equals the same frame rendered by
the per-view calls, and every result is identical alone and in the mix
(continuous batching across headsets, streams and launches)."""
import sys
import time

import numpy as np
import pytest

from paper_2503_23410_amd import inputs as I
from paper_2503_23410_amd import serving

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_23410_amd import vafr as V
    V.load()
    return torch, V


@pytest.fixture(scope="module")
def rig(env):
    """Four headsets over two resident scenes with two display sizes,
    path-traced LP shading (1 sample, 2 bounces)."""
    torch, V = env
    s1 = V.Scene(*I.make_scene("terrain1m"))
    s2 = V.Scene(*I.terrain_scene(256, 128, 64, seed=7))
    layouts = [V.Layout.vafr(V.display(1280, 720)), V.Layout.vafr(V.display(1920, 1080))]
    sh = V.shading(mode=V.VAFR_SHADE_PATH, bounces=2, seed=99)
    heads = []
    for h in range(4):
        cl, cr = I.binocular_cameras()
        heads.append(dict(scene=(s1, s2)[h % 2], layout=layouts[h // 2], cams=(V.camera(cl), V.camera(cr))))
    return dict(V=V, sh=sh, heads=heads, keep=(s1, s2, layouts))


def _server(V, rig, **kw):
    # the watchdog is on in every served test: real launches must never trip it
    args = dict(max_views_per_launch=16, max_inflight=3, n_streams=2, max_queue=256, hbm_budget_bytes=16 << 30,
                watchdog_ms=5000.0)
    args.update(kw)
    s = V.Server(**args)
    for h in rig["heads"]:
        s.add_headset(h["scene"], h["layout"], h["cams"][0], h["cams"][1], rig["sh"])
    return s


def _copy_result(torch, V, rig, r):
    L = rig["heads"][r["headset"]]["layout"]
    imgs = []
    for e in range(2):
        img = torch.empty((L.width * L.height, 4), device="cuda")
        lp = torch.empty((L.n_texels, 4), device="cuda")
        V.copy_from_device(img, r["img"][e])
        V.copy_from_device(lp, r["lp"][e])
        imgs.append((lp, img))
    return imgs


def _gaze(h, f, L):
    g = I.gaze_trace(64, L.width, L.height, seed=70 + h)[f]
    return float(g[0]), float(g[1])


def test_served_frame_equals_direct_calls(env, rig):
    torch, V = env
    s = _server(V, rig)
    h, f = 1, 5
    head = rig["heads"][h]
    L = head["layout"]
    gz = _gaze(h, f, L)
    assert s.submit(h, f, V.gaze(*gz))
    s.wait_idle(30000)
    (r,) = s.poll()
    assert r["status"] == 0
    got = _copy_result(torch, V, rig, r)
    s.release(r["slot"])
    for e in range(2):
        sh = V.shading(mode=V.VAFR_SHADE_PATH, bounces=2, seed=99, frame=f, view=2 * h + e)
        lp = torch.empty((L.n_texels, 4), device="cuda")
        img = torch.empty((L.width * L.height, 4), device="cuda")
        V.vafr_shade_lp(head["scene"], head["cams"][e], V.gaze(*gz), sh, L, lp)
        V.vafr_reconstruct(L, V.gaze(*gz), lp, img)
        torch.cuda.synchronize()
        assert torch.equal(got[e][0], lp) and torch.equal(got[e][1], img)
    s.close()


def test_results_identical_alone_and_in_the_mix(env, rig):
    """32 requests (4 headsets x 8 frames): first each alone, then all
    submitted together so that they share launches and overlap on two
    streams; every LP buffer and image must be bit-identical."""
    torch, V = env
    reqs = [(h, f) for f in range(8) for h in range(4)]
    s = _server(V, rig)
    alone = {}
    for h, f in reqs:
        assert s.submit(h, f, V.gaze(*_gaze(h, f, rig["heads"][h]["layout"])))
        s.wait_idle(30000)
        (r,) = s.poll()
        assert r["status"] == 0
        alone[(h, f)] = _copy_result(torch, V, rig, r)
        s.release(r["slot"])
    st0 = s.stats()
    assert st0["launches"] == 32
    for h, f in reqs:
        assert s.submit(h, f, V.gaze(*_gaze(h, f, rig["heads"][h]["layout"])))
    s.wait_idle(60000)
    mixed = s.poll()
    st = s.stats()
    assert len(mixed) == 32 and all(r["status"] == 0 for r in mixed)
    assert st["launches"] - st0["launches"] < 32            # requests shared launches
    for r in mixed:
        got = _copy_result(torch, V, rig, r)
        ref = alone[(r["headset"], r["frame"])]
        for e in range(2):
            assert torch.equal(got[e][0], ref[e][0]), f"LP of {r['headset'], r['frame']} eye {e} differs"
            assert torch.equal(got[e][1], ref[e][1]), f"image of {r['headset'], r['frame']} eye {e} differs"
        s.release(r["slot"])
    log(f"32 requests alone ({st0['launches']} launches) == in the mix ({st['launches'] - st0['launches']} launches)")
    s.close()


def test_poisson_serving_smoke(env, rig):
    """Half a second of 4 headsets at 90 Hz: every request completes and the
    latency statistics are recorded."""
    torch, V = env
    s = _server(V, rig)
    arr = serving.arrival_times(4, 90.0, 0.5, seed_base=5)
    gazes = [I.gaze_trace(400, h["layout"].width, h["layout"].height, seed=80 + i) for i, h in enumerate(rig["heads"])]
    recs, refused, wall = serving.run(s, V, gazes, arr)
    lat = serving.latency_stats(recs)
    st = s.stats()
    log(f"poisson smoke: {len(arr)} requests, {lat}, launches {st['launches']}, refused {refused}")
    assert refused == 0 and lat["completed"] == len(arr) and st["stalled"] == 0
    s.close()


def test_frame_budget_holds_on_device(env, rig):
    """Four headsets requesting 240 frames/s each (beyond what the device
    renders): with an 11.1 ms budget every served frame completes within it,
    once the device-time model has seen a few launches; the rest is dropped
    as late or replaced, and nothing waits in a growing queue."""
    torch, V = env
    s = _server(V, rig, max_inflight=2, n_streams=1, frame_budget_ms=11.1, latest_only=True)
    gazes = [I.gaze_trace(600, h["layout"].width, h["layout"].height, seed=80 + k) for k, h in enumerate(rig["heads"])]
    warm = serving.arrival_times(4, 240.0, 0.3, seed_base=11)       # the model learns the device times
    serving.run(s, V, gazes, warm)
    st0 = s.stats()
    arr = serving.arrival_times(4, 240.0, 1.0, seed_base=21)
    recs, refused, wall = serving.run(s, V, gazes, arr)
    st = s.stats()
    lat = serving.latency_stats(recs)
    late, sup = st["late"] - st0["late"], st["superseded"] - st0["superseded"]
    log(f"frame budget on device: {lat}, late={late} superseded={sup} refused={refused} "
        f"launches={st['launches'] - st0['launches']}")
    assert refused == 0
    assert lat["completed"] + late + sup == len(arr)
    assert lat["completed"] > 50
    assert lat["p99_ms"] <= 11.1
    assert st["stalled"] == 0
    s.close()
