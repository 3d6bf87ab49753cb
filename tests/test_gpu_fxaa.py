"""GPU parity of the LP anti-aliasing (Sec. 3.4) against the oracle: the
same LP buffer in, every texel out compared (the two follow one stated FP32
operation order), and the whole frame shade -> anti-alias -> inverse map."""
import sys

import numpy as np
import pytest

from paper_2503_23410_amd import inputs as I

pytestmark = pytest.mark.gpu
COLOR_TOL = 2e-3


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


def _fxaa_gpu(torch, V, L, lp_np):
    lp = torch.from_numpy(np.ascontiguousarray(lp_np, np.float32)).cuda()
    out = torch.full_like(lp, -1.0)
    V.vafr_fxaa_lp(L, lp, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _fxaa_window(layout, flagged):
    """Output texels whose anti-aliasing can read one of the `flagged` input
    texels.  Texel (i, j) of column i (n_i rows, angle t = (j + 1/2)/n_i
    turns) reads columns i - 8 .. i + 8 only (radial end search up to 8
    columns, clamped toward i), and in column c only rows within one row
    spacing 1/n_c of an angle it samples; it samples its own and the
    adjacent columns at up to t +- 8/n_i (angular end search) and the other
    columns at t and t +- 1/n_i.  So it can read texel (c, j') only if
    |c - i| <= 8 and the circular angular distance of j' from t is at most
    8/n_i + 1/n_c; half a row of slack on each side covers the FP32
    rounding of the sampled angles."""
    n_rows, col_off = layout.n_rows.astype(np.int64), layout.col_off.astype(np.int64)
    out = np.zeros(layout.n_texels, bool)
    for k in flagged:
        c = int(np.searchsorted(col_off, k, side="right") - 1)
        tc = (k - col_off[c] + 0.5) / n_rows[c]
        for i in range(max(0, c - 8), min(layout.n_cols, c + 9)):
            n = n_rows[i]
            reach = (8.5 / n + 1.5 / n_rows[c]) * n          # in rows of column i
            centre = tc * n - 0.5
            j = np.arange(int(np.floor(centre - reach)), int(np.ceil(centre + reach)) + 1)
            out[col_off[i] + np.mod(j, n)] = True
    return out


def test_fxaa_random_and_shaded_lp_match_oracle(env, O, layout):
    torch, V = env
    W, H = 1920, 1080
    L = V.Layout.vafr(V.display(W, H))
    # random colours: contrast everywhere, every branch of the method
    r = I.random_lp(layout.n_texels, seed=404)
    g = _fxaa_gpu(torch, V, L, r)
    o = O.fxaa_lp(layout, r)
    err = np.abs(g - o).max()
    log(f"fxaa random LP: max_err={err:.2e} changed={np.mean(np.any(o != r, axis=1)):.3f}")
    assert err <= COLOR_TOL
    # a shaded LP buffer of the 1.13M-triangle scene
    v, f = I.make_scene("terrain1m")
    sc = V.Scene(v, f)
    lp = torch.empty((L.n_texels, 4), device="cuda")
    V.vafr_shade_lp(sc, V.camera(I.terrain_camera()), V.gaze(800.0, 500.0), V.shading(), L, lp)
    torch.cuda.synchronize()
    s = lp.cpu().numpy()
    g = _fxaa_gpu(torch, V, L, s)
    o = O.fxaa_lp(layout, s)
    err = np.abs(g - o).max()
    log(f"fxaa shaded LP: max_err={err:.2e} changed={np.mean(np.any(o != s, axis=1)):.3f} "
        f"bit_equal={np.mean(np.all(g == o, axis=1)):.6f}")
    assert err <= COLOR_TOL


def test_fxaa_frame_matches_oracle(env, O, layout):
    """Shade (GPU), anti-alias, inverse-map; the oracle anti-aliases and
    inverse-maps its own shading of the same texels."""
    torch, V = env
    W, H = 640, 360
    g_sc_v, g_sc_f = I.soup_scene()
    sc = V.Scene(g_sc_v, g_sc_f)
    osc = O.Scene(g_sc_v, g_sc_f)
    L = V.Layout.vafr(V.display(W, H))
    gz = (300.0, 200.0)
    lp = torch.empty((L.n_texels, 4), device="cuda")
    aa = torch.empty_like(lp)
    img = torch.empty((W * H, 4), device="cuda")
    V.vafr_shade_lp(sc, V.camera(I.soup_camera()), V.gaze(*gz), V.shading(), L, lp)
    V.vafr_fxaa_lp(L, lp, aa)
    V.vafr_reconstruct(L, V.gaze(*gz), aa, img)
    torch.cuda.synchronize()
    o_lp, o_id, o_fl = O.shade_vafr_texels(osc, layout, np.arange(layout.n_texels), W, H, I.FOV, gz,
                                           I.soup_camera(), O.shading_params())
    o_aa = O.fxaa_lp(layout, o_lp)
    # a flagged texel may hold the other triangle's colour, and FXAA spreads
    # it over the texels whose window reads it: compare every other texel
    g_aa = aa.cpu().numpy()
    affected = _fxaa_window(layout, np.nonzero(o_fl)[0])
    diff = np.abs(g_aa - o_aa).max(axis=1)
    log(f"fxaa frame: flagged texels={int(o_fl.sum())} in their windows={int(affected.sum())} "
        f"max LP err outside={diff[~affected].max():.2e}")
    assert o_fl.sum() <= 1e-4 * layout.n_texels
    assert diff[~affected].max() <= COLOR_TOL
    p = O.film_pitch(W, H, *I.FOV)
    pix = np.arange(W * H)
    ref, pf = O.vafr_reconstruct(layout, o_aa, W, H, p, O.gaze_film(W, H, p, *gz), pix, affected.astype(np.uint8))
    err = np.abs(img.cpu().numpy() - ref).max(axis=1)
    ok = ~pf
    log(f"fxaa frame image: max_err={err[ok].max():.2e} over {int(ok.sum())} pixels ({int(pf.sum())} excluded)")
    assert err[ok].max() <= COLOR_TOL


def test_fxaa_rejects_bad_calls(env):
    torch, V = env
    L = V.Layout.vafr(V.display(64, 64))
    lp = torch.zeros((L.n_texels, 4), device="cuda")
    with pytest.raises(V.VafrError) as ei:
        V.vafr_fxaa_lp(L, lp, lp)                                  # in place
    assert ei.value.code == V.VAFR_E_ARG
    LM = V.Layout.lmfr(V.display(64, 64), 1.8, 4.0)
    with pytest.raises(V.VafrError) as ei:
        V.vafr_fxaa_lp(LM, lp, torch.zeros_like(lp))
    assert ei.value.code == V.VAFR_E_UNSUPPORTED


@pytest.mark.parametrize("cap,aniso", [(9.0, None), (None, ([0.0, 30.0], [1.0, 0.5])),
                                       (18.0, ([0.0, 10.0, 40.0], [1.0, 0.8, 0.4]))])
def test_fxaa_on_capped_and_anisotropic_layouts(env, O, cap, aniso):
    """The anti-aliasing reads neighbours across columns of different row
    counts; layouts of the device-adapted curves and of anisotropic
    tangential rates change those counts: every texel against the oracle."""
    torch, V = env
    if cap is None:
        ecc, cpd = [0.0, 10.0, 20.0, 30.0, 60.0], [40.0, 10.0, 6.0, 5.0, 4.0]
    else:
        ecc, cpd = V.acuity_capped(cap)
    L = V.Layout.vafr(V.display(1280, 720), ecc, cpd, 60.0, aniso=aniso)
    ref_layout = O.Layout(O.Acuity(ecc, cpd, aniso=aniso), 60.0)
    assert L.n_texels == ref_layout.n_texels
    r = I.random_lp(L.n_texels, seed=405)
    g = _fxaa_gpu(torch, V, L, r)
    o = O.fxaa_lp(ref_layout, r)
    err = np.abs(g - o).max()
    log(f"fxaa cap={cap} aniso={aniso}: texels={L.n_texels} max_err={err:.2e} "
        f"changed={np.mean(np.any(o != r, axis=1)):.3f}")
    assert err <= COLOR_TOL
