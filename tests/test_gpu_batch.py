"""Batched frames (one traversal launch + one reconstruction launch over many
views, optionally replayed from a hipGraph) must give exactly the results
of the per-view calls, which the parity tests pin to the oracle."""
import os
import sys

import numpy as np
import pytest

from paper_2503_23410_amd import inputs as I

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
def scene(env):
    torch, V = env
    v, f = I.make_scene("terrain1m")
    return V.Scene(v, f)


def _views(torch, V, scene, sizes, gazes, cams, kinds):
    """Buffers + per-view descriptors for a mixed batch."""
    out = []
    for (W, H), gz, cam, kind in zip(sizes, gazes, cams, kinds):
        d = V.display(W, H, I.FOV)
        if kind == V.VAFR_VIEW_FULL:
            L = None
            lp = None
        else:
            L = (V.Layout.vafr(d) if kind == V.VAFR_VIEW_VAFR else
                 V.Layout.lmfr(d, 1.8, 4.0) if kind == V.VAFR_VIEW_LMFR else V.Layout.lafr(d, 2.2))
            lp = torch.full((L.n_texels, 4), -1.0, device="cuda")
        n_hit = L.n_texels if L is not None else W * H
        hit = torch.full((n_hit,), -7, device="cuda", dtype=torch.int32)
        img = torch.full((W * H, 4), -1.0, device="cuda")
        out.append(dict(kind=kind, disp=d, layout=L, lp=lp, hit=hit, img=img, gaze=V.gaze(*gz), cam=V.camera(cam)))
    return out


def _run_individual(V, scene, vs, sh):
    for w in vs:
        if w["kind"] == V.VAFR_VIEW_FULL:
            V.full_shade(scene, w["cam"], w["disp"], sh, w["img"], w["hit"])
        elif w["kind"] == V.VAFR_VIEW_VAFR:
            V.vafr_shade_lp(scene, w["cam"], w["gaze"], sh, w["layout"], w["lp"], w["hit"])
            V.vafr_reconstruct(w["layout"], w["gaze"], w["lp"], w["img"])
        elif w["kind"] == V.VAFR_VIEW_LMFR:
            V.lmfr_shade_lp(scene, w["cam"], w["gaze"], sh, w["layout"], w["lp"], w["hit"])
            V.lmfr_reconstruct(w["layout"], w["gaze"], w["lp"], w["img"])
        else:
            V.lafr_shade_lp(scene, w["cam"], w["gaze"], sh, w["layout"], w["lp"], w["hit"])
            V.lafr_reconstruct(w["layout"], w["gaze"], w["lp"], w["img"])


def _descs(V, scene, vs, sh):
    return [V.view(w["kind"], scene, w["cam"], w["gaze"], sh, layout=w["layout"], disp=w["disp"], lp_rgba=w["lp"],
                   hit_id=w["hit"], img_rgba=w["img"]) for w in vs]


def _snapshot(vs):
    return [(None if w["lp"] is None else w["lp"].clone(), w["hit"].clone(), w["img"].clone()) for w in vs]


def _clear(torch, vs):
    for w in vs:
        if w["lp"] is not None:
            w["lp"].fill_(-1.0)
        w["hit"].fill_(-7)
        w["img"].fill_(-1.0)


def _assert_equal(torch, ref, vs, what):
    for i, (w, (lp, hit, img)) in enumerate(zip(vs, ref)):
        if lp is not None:
            assert torch.equal(w["lp"], lp), f"{what}: view {i} LP differs"
        assert torch.equal(w["hit"], hit), f"{what}: view {i} hit ids differ"
        assert torch.equal(w["img"], img), f"{what}: view {i} image differs"


def test_batch_equals_individual_calls(env, scene):
    """16 views of uneven size (sizes drawn from 720p..8K, gaze per view),
    mostly VaFR plus one LMFR, one LaFR(2.2) and one full-resolution view,
    eager and graph."""
    torch, V = env
    sizes, gazes = I.batch_views(16, seed=4)
    kinds = [V.VAFR_VIEW_VAFR] * 16
    kinds[5] = V.VAFR_VIEW_LMFR
    kinds[11] = V.VAFR_VIEW_FULL
    kinds[8] = V.VAFR_VIEW_LAFR
    cams = [I.terrain_camera(0.01 * k) for k in range(16)]
    vs = _views(torch, V, scene, sizes, gazes, cams, kinds)
    sh = V.shading()
    _run_individual(V, scene, vs, sh)
    torch.cuda.synchronize()
    ref = _snapshot(vs)
    for use_graph in (False, True):
        for tb, rows in ((128, 4), (64, 1), (256, 8)):
            _clear(torch, vs)
            b = V.Batch(16, trace_block=tb, recon_rows=rows, use_graph=use_graph)
            b.run(_descs(V, scene, vs, sh))
            torch.cuda.synchronize()
            _assert_equal(torch, ref, vs, f"graph={use_graph} block={tb} rows={rows}")
            b.close()
    log("batch of 16 views equals the per-view calls (eager and graph)")


@pytest.mark.parametrize("rows", [1, 4, 8])
def test_paired_reconstruction_equals_individual_calls(env, scene, rows):
    """VaFR views that share one layout object and one gaze (binocular eyes)
    are reconstructed in shared workgroups.  Views: a pair on a ragged
    1000x563 display; a pair plus a third view with the same gaze (it stays
    single, since a descriptor holds one partner); a view with its own gaze;
    an LMFR view between them.  Every image, LP buffer and hit id equals the
    per-view calls bit for bit, eager and graph, at every tile height."""
    torch, V = env
    d1, d2 = V.display(1000, 563, I.FOV), V.display(1920, 1080, I.FOV)
    L1, L2 = V.Layout.vafr(d1), V.Layout.vafr(d2)
    Lm = V.Layout.lmfr(d2, 1.8, 4.0)
    cl, cr = I.binocular_cameras()
    specs = [(V.VAFR_VIEW_VAFR, d1, L1, (420.5, 300.25), cl), (V.VAFR_VIEW_VAFR, d1, L1, (420.5, 300.25), cr),
             (V.VAFR_VIEW_VAFR, d2, L2, (700.0, 500.0), cl), (V.VAFR_VIEW_VAFR, d2, L2, (700.0, 500.0), cr),
             (V.VAFR_VIEW_VAFR, d2, L2, (700.0, 500.0), I.terrain_camera(0.05)),
             (V.VAFR_VIEW_LMFR, d2, Lm, (700.0, 500.0), cl),
             (V.VAFR_VIEW_VAFR, d2, L2, (-50.0, 1200.0), cr)]
    vs = []
    for kind, d, L, gz, cam in specs:
        vs.append(dict(kind=kind, disp=d, layout=L, lp=torch.full((L.n_texels, 4), -1.0, device="cuda"),
                       hit=torch.full((L.n_texels,), -7, device="cuda", dtype=torch.int32),
                       img=torch.full((d.width * d.height, 4), -1.0, device="cuda"), gaze=V.gaze(*gz),
                       cam=V.camera(cam)))
    sh = V.shading()
    _run_individual(V, scene, vs, sh)
    torch.cuda.synchronize()
    ref = _snapshot(vs)
    for use_graph in (False, True):
        b = V.Batch(8, trace_block=128, recon_rows=rows, use_graph=use_graph)
        for rep in range(2):
            _clear(torch, vs)
            b.run(_descs(V, scene, vs, sh))
            torch.cuda.synchronize()
            _assert_equal(torch, ref, vs, f"rows={rows} graph={use_graph} run {rep}")
        b.close()


def test_largest_batch_equals_individual_calls(env, scene):
    """The batch's limit of 256 views, on small displays (1x1 to 97x61):
    VaFR views in binocular pairs (shared layout and gaze), single VaFR
    views with their own gaze, LMFR and full-resolution views (displays of
    33x17 and up), eager and graph; every output equals the per-view calls
    bit for bit, and a 257th view is refused."""
    torch, V = env
    rng = np.random.default_rng(256)
    sizes = [(1, 1), (7, 5), (33, 17), (64, 16), (97, 61)]
    layouts = {sz: V.Layout.vafr(V.display(sz[0], sz[1], I.FOV)) for sz in sizes}
    cl, cr = I.binocular_cameras()
    vs = []
    while len(vs) < 256:
        W, H = sizes[int(rng.integers(len(sizes)))]
        d = V.display(W, H, I.FOV)
        gz = (float(rng.uniform(-0.2, 1.2) * W), float(rng.uniform(-0.2, 1.2) * H))
        kind = int(rng.choice([V.VAFR_VIEW_VAFR, V.VAFR_VIEW_VAFR, V.VAFR_VIEW_LMFR, V.VAFR_VIEW_FULL]))
        if W * H < 33 * 17:
            kind = V.VAFR_VIEW_VAFR                  # the LMFR map needs a few pixels of extent
        pair = kind == V.VAFR_VIEW_VAFR and len(vs) < 255 and rng.random() < 0.6
        for cam in ((cl, cr) if pair else (I.terrain_camera(float(rng.uniform(0.0, 0.1))),)):
            L = (layouts[(W, H)] if kind == V.VAFR_VIEW_VAFR else
                 V.Layout.lmfr(d, 1.8, 4.0) if kind == V.VAFR_VIEW_LMFR else None)
            n = L.n_texels if L is not None else W * H
            vs.append(dict(kind=kind, disp=d, layout=L,
                           lp=None if L is None else torch.full((L.n_texels, 4), -1.0, device="cuda"),
                           hit=torch.full((n,), -7, device="cuda", dtype=torch.int32),
                           img=torch.full((W * H, 4), -1.0, device="cuda"), gaze=V.gaze(*gz), cam=V.camera(cam)))
    assert len(vs) == 256
    sh = V.shading()
    _run_individual(V, scene, vs, sh)
    torch.cuda.synchronize()
    ref = _snapshot(vs)
    for use_graph in (False, True):
        b = V.Batch(256, use_graph=use_graph)
        for rep in range(2):
            _clear(torch, vs)
            b.run(_descs(V, scene, vs, sh))
            torch.cuda.synchronize()
            _assert_equal(torch, ref, vs, f"256 views graph={use_graph} run {rep}")
        with pytest.raises(V.VafrError):
            b.run(_descs(V, scene, vs + vs[:1], sh))
        b.close()


def test_graph_cache_evicts_and_rebuilds_launch_shapes(env, scene):
    """More launch shapes than the batch keeps as graphs (32): 40 frames of
    two views on displays of different sizes, then the first shapes again
    after they were evicted, all run back to back (up to four frames in
    flight while shapes are evicted); every frame equals the per-view calls
    bit for bit."""
    torch, V = env
    sh = V.shading()
    cl, cr = I.binocular_cameras()
    sizes = [(40 + 7 * k, 24 + 5 * k) for k in range(40)]
    frames = list(range(40)) + [0, 1, 2, 39]
    per_frame = []
    for k in frames:
        W, H = sizes[k]
        vs = _views(torch, V, scene, [(W, H)] * 2, [(0.4 * W, 0.6 * H)] * 2, [cl, cr],
                    [V.VAFR_VIEW_VAFR, V.VAFR_VIEW_VAFR])
        _run_individual(V, scene, vs, sh)
        per_frame.append(vs)
    torch.cuda.synchronize()
    refs = [_snapshot(vs) for vs in per_frame]
    for vs in per_frame:
        _clear(torch, vs)
    b = V.Batch(2, trace_block=128, recon_rows=4, use_graph=True)
    for vs in per_frame:
        b.run(_descs(V, scene, vs, sh))
    torch.cuda.synchronize()
    for f, (vs, ref) in enumerate(zip(per_frame, refs)):
        _assert_equal(torch, ref, vs, f"frame {f} (shape {frames[f]})")
    b.close()


def test_null_config_gives_the_documented_defaults(env):
    """vafr_batch_create with a NULL configuration: trace_block 128,
    recon_rows 4, use_graph 1, as the header states."""
    import ctypes as C
    torch, V = env
    lib = V.load()
    h = C.c_void_p()
    assert lib.vafr_batch_create(2, None, C.byref(h)) == V.VAFR_OK
    c = V.vafr_batch_config()
    assert lib.vafr_batch_get_config(h, C.byref(c)) == V.VAFR_OK
    lib.vafr_batch_destroy(h)
    assert (c.trace_block, c.recon_rows, c.use_graph) == (128, 4, 1)


def test_graph_replays_track_parameter_updates(env, scene):
    """Replay the captured frame with new gazes and cameras each time, with
    eager work between replays; every replay equals the eager result."""
    torch, V = env
    sizes = [(1920, 1080), (1280, 720), (1920, 1080)]
    kinds = [V.VAFR_VIEW_VAFR, V.VAFR_VIEW_VAFR, V.VAFR_VIEW_LMFR]
    trace = I.gaze_trace(12, 1920, 1080, seed=30)
    b = V.Batch(4, use_graph=True)
    sh = V.shading()
    for f in range(5):
        gz = [tuple(trace[2 * f]), tuple(trace[2 * f + 1] * 0.66), tuple(trace[2 * f + 2])]
        cams = [I.terrain_camera(0.02 * f + 0.01 * k) for k in range(3)]
        vs = _views(torch, V, scene, sizes, gz, cams, kinds)
        _run_individual(V, scene, vs, sh)
        torch.cuda.synchronize()
        ref = _snapshot(vs)
        _clear(torch, vs)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()                       # unrelated eager work between replays
        b.run(_descs(V, scene, vs, sh))
        torch.cuda.synchronize()
        _assert_equal(torch, ref, vs, f"replay {f}")
    b.close()


def test_planned_dispatch_keeps_results_over_frames(env, scene):
    """From the second frame on, the batched traversal dispatches each XCD's
    workgroups longest-first by the previous frame's durations; every frame
    must still equal the per-view calls (each block traced exactly once),
    eager and graph, with the gaze moving between frames."""
    torch, V = env
    sizes = [(3840, 2160), (3840, 2160)]
    kinds = [V.VAFR_VIEW_VAFR, V.VAFR_VIEW_VAFR]
    trace = I.gaze_trace(8, 3840, 2160, seed=31)
    cl, cr = I.binocular_cameras()
    sh = V.shading()
    for use_graph in (False, True):
        b = V.Batch(2, trace_block=128, recon_rows=8, use_graph=use_graph)
        for f in range(4):
            gz = [tuple(trace[f]), tuple(trace[f])]
            vs = _views(torch, V, scene, sizes, gz, [cl, cr], kinds)
            _run_individual(V, scene, vs, sh)
            torch.cuda.synchronize()
            ref = _snapshot(vs)
            _clear(torch, vs)
            b.run(_descs(V, scene, vs, sh))
            torch.cuda.synchronize()
            _assert_equal(torch, ref, vs, f"graph={use_graph} frame {f}")
        b.close()


def test_autotune_picks_a_valid_shape(env, scene):
    torch, V = env
    sizes, gazes = I.batch_views(6, seed=8)
    kinds = [V.VAFR_VIEW_VAFR] * 6
    vs = _views(torch, V, scene, sizes, gazes, [I.terrain_camera()] * 6, kinds)
    sh = V.shading()
    _run_individual(V, scene, vs, sh)
    torch.cuda.synchronize()
    ref = _snapshot(vs)
    b = V.Batch(8)
    cfg = b.autotune(_descs(V, scene, vs, sh), reps=2)
    log(f"autotuned shape: {cfg}")
    assert cfg["trace_block"] in (64, 128, 256) and cfg["recon_rows"] in (1, 2, 4, 8)
    assert b.config() == cfg
    _clear(torch, vs)
    b.run(_descs(V, scene, vs, sh))
    torch.cuda.synchronize()
    _assert_equal(torch, ref, vs, "after autotune")
    b.close()


def test_batch_rejects_bad_views(env, scene):
    torch, V = env
    b = V.Batch(2)
    L = V.Layout.vafr(V.display(64, 64))
    lp = torch.empty((L.n_texels, 4), device="cuda")
    good = V.view(V.VAFR_VIEW_VAFR, scene, V.camera(I.terrain_camera()), V.gaze(1.0, 1.0), V.shading(), layout=L,
                  lp_rgba=lp)
    with pytest.raises(V.VafrError):
        b.run([good, good, good])                       # more than max_views
    bad = V.view(V.VAFR_VIEW_VAFR, scene, V.camera(I.terrain_camera()), V.gaze(1.0, 1.0), V.shading(), layout=L)
    with pytest.raises(V.VafrError):
        b.run([bad])                                    # no LP buffer
    b.run([good])
    torch.cuda.synchronize()
    b.close()


# 6 cases by default; VAFR_BATCH_CASES asks for more, for a longer sweep by hand.
N_BATCH_CASES = int(os.environ.get("VAFR_BATCH_CASES", "6"))


@pytest.mark.parametrize("case", range(N_BATCH_CASES))
def test_random_batches_equal_individual_calls(env, scene, case):
    """Seeded random batches: 1-12 views of random kind (VaFR, LMFR, full
    resolution), display size (1-900 px per side), gaze (on and off
    screen), camera and scene (the terrain and a small soup in one batch),
    one shading per batch (Lambert, no shadows, or path mode), random launch
    shape, eager or graph; a VaFR view followed by another becomes a
    binocular pair (shared layout, display and gaze) half of the time, so
    the two share reconstruction workgroups.  Each batch runs twice (the
    second run follows the dispatch plan the first one recorded) and must
    equal the per-view calls bit for bit."""
    torch, V = env
    rng = np.random.default_rng(900 + case)
    sv, sf = I.soup_scene()
    soup = V.Scene(sv, sf)
    n = int(rng.integers(1, 13))
    kinds = [int(rng.choice([V.VAFR_VIEW_VAFR, V.VAFR_VIEW_LMFR, V.VAFR_VIEW_FULL], p=[0.6, 0.2, 0.2]))
             for _ in range(n)]
    sizes = [(int(rng.integers(1, 901)), int(rng.integers(1, 901))) for _ in range(n)]
    gazes = [(float(rng.uniform(-0.2, 1.2) * w), float(rng.uniform(-0.2, 1.2) * h)) for w, h in sizes]
    cams = [I.terrain_camera(float(rng.uniform(-0.05, 0.05))) for _ in range(n)]
    scenes = [scene if rng.uniform() < 0.7 else soup for _ in range(n)]
    mode = case % 3
    if mode == 2:
        sh = V.shading(mode=V.VAFR_SHADE_PATH, bounces=int(rng.integers(0, 3)), frame=case, seed=77 + case)
    else:
        sh = V.shading(shadow=mode == 0)
    pair = [False] + [kinds[i - 1] == kinds[i] == V.VAFR_VIEW_VAFR and rng.uniform() < 0.5 for i in range(1, n)]
    for i in range(1, n):
        if pair[i] and not pair[i - 1]:
            sizes[i], gazes[i] = sizes[i - 1], gazes[i - 1]
        else:
            pair[i] = False
    vs = _views(torch, V, scene, sizes, gazes, cams, kinds)
    for i in range(1, n):
        if pair[i]:
            vs[i]["layout"] = vs[i - 1]["layout"]
    for w, sc in zip(vs, scenes):
        w["scene"] = sc
    for w in vs:
        _run_individual(V, w["scene"], [w], sh)
    torch.cuda.synchronize()
    ref = _snapshot(vs)
    tb = int(rng.choice([64, 128, 256]))
    rows = int(rng.choice([1, 2, 4, 8]))
    use_graph = bool(rng.integers(0, 2))
    b = V.Batch(12, trace_block=tb, recon_rows=rows, use_graph=use_graph)
    descs = [V.view(w["kind"], w["scene"], w["cam"], w["gaze"], sh, layout=w["layout"], disp=w["disp"],
                    lp_rgba=w["lp"], hit_id=w["hit"], img_rgba=w["img"]) for w in vs]
    for rep in range(2):
        _clear(torch, vs)
        b.run(descs)
        torch.cuda.synchronize()
        _assert_equal(torch, ref, vs, f"case {case} run {rep} (views {n}, block {tb}, rows {rows}, graph {use_graph})")
    b.close()
    log(f"random batch {case}: {n} views {kinds} ({sum(pair)} pairs) mode {mode} block {tb} rows {rows} "
        f"graph {use_graph}: equal")


@pytest.mark.parametrize("bounces", [(2, 2, 2), (3, 3, 3), (0, 0, 0), (1, 1, 1), (8, 8, 8), (2, 0, 3)])
def test_phased_path_mode_equals_single_pass(env, scene, bounces):
    """Batched path-mode views run in phases (bounce 0 in the traversal
    launch, each later bounce in a launch over the compacted list of live
    paths, path state in memory between launches); the per-view calls run
    each path in one pass.  Both must agree bit for bit: VaFR, LMFR and
    full-resolution path-mode views (bounce counts per view as given) plus a
    Lambert view in one batch, eager and graph, three frames in a row (graph
    replays with new gazes)."""
    torch, V = env
    sizes = [(1280, 720), (640, 480), (301, 177), (1920, 1080)]
    kinds = [V.VAFR_VIEW_VAFR, V.VAFR_VIEW_LMFR, V.VAFR_VIEW_FULL, V.VAFR_VIEW_VAFR]
    cams = [I.terrain_camera(0.01 * k) for k in range(4)]
    shs = [V.shading(mode=V.VAFR_SHADE_PATH, bounces=bn, frame=3, view=k, seed=99) for k, bn in enumerate(bounces)]
    shs.append(V.shading())
    for use_graph in (False, True):
        b = V.Batch(8, trace_block=128, recon_rows=4, use_graph=use_graph)
        for frame in range(3):
            gazes = [(0.3 * w + 40.0 * frame, 0.6 * h - 25.0 * frame) for w, h in sizes]
            vs = _views(torch, V, scene, sizes, gazes, cams, kinds)
            for w, sh in zip(vs, shs):
                w["sh"] = sh
                _run_individual(V, scene, [w], sh)
            torch.cuda.synchronize()
            ref = _snapshot(vs)
            _clear(torch, vs)
            b.run([V.view(w["kind"], scene, w["cam"], w["gaze"], w["sh"], layout=w["layout"], disp=w["disp"],
                          lp_rgba=w["lp"], hit_id=w["hit"], img_rgba=w["img"]) for w in vs])
            torch.cuda.synchronize()
            _assert_equal(torch, ref, vs, f"bounces {bounces} graph {use_graph} frame {frame}")
        b.close()
    log(f"phased path mode (bounces {bounces}) equals the single pass (eager and graph, 3 frames)")
