"""Seeded random parity sweep: the HIP path against the oracle on scenes,
cameras, fields of view, display sizes, gazes and shading modes drawn at
random (outside the fixed configurations).

Each case compares, through the C ABI:
  - LP texels (a seeded sample): hit ids exact and colours within 2e-3 on
    rays the oracle does not flag as near ties;
  - the inverse map of the GPU's own LP buffer onto every display pixel
    against the oracle's inverse map of the same buffer;
  - the full-resolution ray cast on every display pixel.
Random soups hold long thin, tiny and degenerate triangles; flagged rays are
reported and kept to at most 1e-4 of the compared rays, the stated
tolerance (their result is not unique): per case for the 30 committed
cases, and over all comparisons in any sweep.  A sweep of 300 cases gave
133 flagged of 15.1M outputs (8.8e-6), no hit-id mismatch and colour error
0; eleven of its cases had 3-4 flagged rays in about 30,000 samples, or 1
in a few thousand."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

COLOR_TOL = 2e-3
# 30 cases by default; VAFR_RANDOM_CASES asks for more (seeds continue the
# same sequence), for a longer sweep by hand.
N_CASES = int(os.environ.get("VAFR_RANDOM_CASES", "30"))
N_COMMITTED = 30
# (flagged, outputs) of every comparison, for the aggregate flag rate
_FLAGS = []


@pytest.fixture(scope="module")
def env(O):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_23410_amd import vafr as V
    V.load()
    O.set_threads(16)
    return torch, V


def _case(k):
    rng = np.random.default_rng(7100 + k)
    n = [1, 3, 40, 600, 6000][k % 5]
    centres = rng.uniform(-1.0, 1.0, (n, 1, 3))
    size = 10.0 ** rng.uniform(-1.5, 0.3, (n, 1, 1)) if n > 3 else np.full((n, 1, 1), 1.5)
    v = centres + size * rng.normal(size=(n, 3, 3))
    if n >= 3:
        v[0, 2] = v[0, 1]                      # degenerate: two equal vertices
        v[1, :, 1] = v[1, 0, 1]                # flat in y
        v[2] = [[-3.0, 0.0, 0.0], [3.0, 0.01, 0.0], [0.0, 0.0, 0.02]]   # long and thin
        # a large ground quad under the soup (receives shadows)
        g = -1.6
        quad = np.array([[[-9, g, -9], [9, g, -9], [9, g, 9]], [[-9, g, -9], [9, g, 9], [-9, g, 9]]], np.float64)
        v = np.concatenate([v, quad])
    verts = v.astype(np.float32).reshape(-1, 3)
    tris = np.arange(verts.shape[0], dtype=np.int32).reshape(-1, 3)
    eye = rng.normal(size=3)
    eye[1] = abs(eye[1])                       # above the ground
    eye = eye / np.linalg.norm(eye) * rng.uniform(1.8, 4.0)
    fwd = rng.uniform(-0.3, 0.3, 3) - eye
    fwd /= np.linalg.norm(fwd)
    up0 = rng.normal(size=3)
    right = np.cross(up0, fwd)
    right /= np.linalg.norm(right)
    up = np.cross(fwd, right)
    cam = np.concatenate([eye, right, up, fwd]).astype(np.float32)
    fov = (float(rng.uniform(30.0, 140.0)), float(rng.uniform(30.0, 140.0)))
    W, H = (int(x) for x in rng.integers(1, 360, 2))
    gaze = (float(rng.uniform(-0.2, 1.2) * W), float(rng.uniform(-0.2, 1.2) * H))
    mode = ["lambert", "noshadow", "path"][k % 3]
    bounces = int((k // 3) % 3) if mode == "path" else 0
    seed = int(rng.integers(1, 2 ** 62))
    return verts, tris, cam, fov, W, H, gaze, mode, bounces, seed


def _check(name, g_rgba, g_id, o_rgba, o_id, flag):
    unf = flag == 0
    mism = int(((g_id != o_id) & unf).sum())
    err = np.abs(g_rgba - o_rgba).max(axis=1)
    worst = float(err[unf].max()) if unf.any() else 0.0
    print(f"{name}: n={len(o_id)} mismatches={mism} flagged={int(flag.sum())} max_err={worst:.2e} "
          f"hit_frac={(o_id >= 0).mean():.3f}", flush=True)
    _FLAGS.append((int(flag.sum()), len(flag)))
    assert mism == 0
    assert worst <= COLOR_TOL
    # The 30 committed cases hold each case's flagged rays within 1e-4 of its
    # own sample.  In a longer sweep a case's count is a few rays (1e-4 of a
    # 30,000-texel sample is 3), so the rate bound applies to the total, in
    # test_flag_rate_over_all_cases.
    if N_CASES <= N_COMMITTED:
        assert flag.sum() <= 1e-4 * len(flag), f"{int(flag.sum())} flagged rays exceed 1e-4 of {len(flag)}"


@pytest.mark.parametrize("k", range(N_CASES))
def test_random_case_matches_oracle(env, O, layout, k):
    torch, V = env
    verts, tris, cam, fov, W, H, gaze, mode, bounces, seed = _case(k)
    name = f"case {k} ({len(tris)} tris, {W}x{H}, fov {fov[0]:.0f}x{fov[1]:.0f}, {mode}{bounces or ''})"
    print(name, flush=True)
    g_sc, o_sc = V.Scene(verts, tris), O.Scene(verts, tris)
    disp = V.display(W, H, fov)
    L = V.Layout.vafr(disp)
    if mode == "path":
        sh = V.shading(mode=V.VAFR_SHADE_PATH, bounces=bounces, frame=k, view=1, seed=seed)
    else:
        sh = V.shading(shadow=mode == "lambert")
    osh = O.shading_params(shadow=mode != "noshadow")
    lp = torch.empty((L.n_texels, 4), device="cuda", dtype=torch.float32)
    hid = torch.empty(L.n_texels, device="cuda", dtype=torch.int32)
    V.vafr_shade_lp(g_sc, V.camera(cam), V.gaze(*gaze), sh, L, lp, hid)
    torch.cuda.synchronize()
    rng = np.random.default_rng(k)
    idx = np.unique(rng.integers(0, layout.n_texels, 30000))
    p = O.film_pitch(W, H, *fov)
    G = O.gaze_film(W, H, p, *gaze)
    org, d = O.vafr_rays(layout, idx, G, cam)
    if mode == "path":
        o_rgba, o_id, o_fl = o_sc.shade_path(org, d, idx, osh, seed, k, 1, bounces)
    else:
        o_rgba, o_id, o_fl = o_sc.shade(org, d, osh)
    lp_np = lp.cpu().numpy()
    _check(name + " LP", lp_np[idx], hid.cpu().numpy()[idx], o_rgba, o_id, o_fl)
    # inverse map of the GPU's buffer, every pixel
    img = torch.empty((H * W, 4), device="cuda", dtype=torch.float32)
    V.vafr_reconstruct(L, V.gaze(*gaze), lp, img)
    torch.cuda.synchronize()
    ref, _ = O.vafr_reconstruct(layout, lp_np, W, H, p, G, np.arange(W * H))
    err = float(np.abs(img.cpu().numpy() - ref).max())
    print(f"{name} image: max_err={err:.2e}", flush=True)
    assert err <= COLOR_TOL
    # full resolution, every pixel (Lambert modes)
    if mode != "path":
        fid = torch.empty(H * W, device="cuda", dtype=torch.int32)
        V.full_shade(g_sc, V.camera(cam), disp, sh, img, fid)
        torch.cuda.synchronize()
        f_rgba, f_id, f_fl = O.shade_full_pixels(o_sc, np.arange(W * H), W, H, fov, cam, osh)
        _check(name + " full-res", img.cpu().numpy(), fid.cpu().numpy(), f_rgba, f_id, f_fl)


def test_flag_rate_over_all_cases(env):
    """Flagged rays over every comparison of the sweep stay within 1e-4 of
    all outputs compared (runs after the cases, in file order)."""
    if not _FLAGS:
        pytest.skip("no case ran")
    f = sum(x for x, _ in _FLAGS)
    n = sum(y for _, y in _FLAGS)
    print(f"sweep of {N_CASES} cases: {f} flagged of {n} outputs ({f / n:.2e})", flush=True)
    assert f <= 1e-4 * n
