"""Pins for the oracle's LaFR comparison mapping (Sec. 4.1 Eq. (15)) and the
LMFR shading rate (Eq. (16)).

The paper prints the mapping u_LaFR(z) (Eq. (15)) and, separately, its
derivative as a shading rate (Eq. (17), for beta = 0.7); the same for LMFR
(Eq. (14) and Eq. (16)).  A numerical derivative of the oracle's forward map
checked against the printed closed forms fixes each piece of the map: a
dropped factor, a wrong sign or a swapped Z_ef would show up there.  Fa is a
reading of a garbled formula (the printed one has no real value for a = 4);
its value is parity unpinned, and only its definedness and the qualitative
behaviour the paper describes (a shading-rate jump at the foveal boundary)
are checked.
"""
import math

import numpy as np
import pytest

DISPLAYS = {"2K": (2560, 1440), "8K": (7680, 4320)}


def _lw(e_deg, w, lnL):
    """LW(e) of Sec. 4.1: w pi / (180 ln L sin e cos e)."""
    e = np.radians(e_deg)
    return w * math.pi / (180.0 * lnL * np.sin(e) * np.cos(e))


def _u_at_ecc(O, W, H, p, g, w, h, e_deg, fn):
    """u of the point at eccentricity e straight below the gaze point
    (vertical film pitch p[1], the paper's c_r)."""
    r = np.tan(np.radians(e_deg)) / p[1]
    xy = np.stack([np.full_like(r, g[0]), g[1] + r], 1)
    return fn(xy)


def _numeric_sr(O, W, H, p, g, w, h, e_deg, fn, de=1e-4):
    up = _u_at_ecc(O, W, H, p, g, w, h, e_deg + de, fn)
    um = _u_at_ecc(O, W, H, p, g, w, h, e_deg - de, fn)
    return 0.5 * (up - um) / (2.0 * de)


@pytest.mark.parametrize("name", sorted(DISPLAYS))
@pytest.mark.parametrize("gaze_frac", [(0.5, 0.5), (0.3, 0.2)])
def test_lafr_shading_rate_matches_eq17(O, paper, name, gaze_frac):
    """0.5 du/de of the oracle's Eq. (15) equals the printed Eq. (17) on both
    sides of the foveal boundary (beta = 0.7, as Eq. (17) assumes), the
    second piece up to the factor 2 it prints without."""
    lp = paper["lafr_parameters"]
    W, H = DISPLAYS[name]
    w, h = O.lmfr_dims(W, H, lp["original"]["delta"])
    p = O.film_pitch(W, H)
    g = (gaze_frac[0] * W, gaze_frac[1] * H)
    alpha, beta = lp["original"]["alpha"], lp["original"]["beta"]
    assert beta == lp["beta_reference"]
    lnL, Zef, Fa, Uef = O.lafr_consts(W, H, p, g[0], g[1], O.LAFR_A, alpha)
    # eccentricities that stay on screen below the gaze point
    e_hi = math.degrees(math.atan((H - g[1] - 2.0) * p[1]))
    e = np.concatenate([np.linspace(0.8, 4.7, 12), np.linspace(5.1, min(50.0, e_hi - 0.5), 24)])

    def fwd(xy):
        return O.lafr_forward(W, H, p, g[0], g[1], w, h, xy, O.LAFR_A, alpha, beta)[0]

    sr = _numeric_sr(O, W, H, p, g, w, h, e, fwd)
    z = np.log(np.tan(np.radians(e)) / p[1]) / lnL
    lw = _lw(e, w, lnL)
    fov = e <= lp["foveal_boundary_deg"]
    sr1 = (1 - Fa) / (2 * Fa) * (z - z * Fa) ** ((1 - Fa) / Fa) * lw
    zo = np.where(fov, 1.0, z)          # second piece evaluated outside the fovea only
    za = (1 / zo - 1 / Zef) / (1 / Zef - 1)
    sr2 = 2 * (1 - Uef) / (-math.pi * np.sqrt(1 - za ** 2 + fov)) * (1 / (1 / Zef - 1)) * (-1 / zo ** 2) * lw
    # The printed second piece is du/de, not 0.5 du/de: it lacks the 1/2 of
    # Eq. (13) that its first piece and Eq. (16) carry.  Eq. (15) is the
    # definition, so the second piece is compared with half the printed form.
    ref = np.where(fov, sr1, 0.5 * sr2)
    assert np.all(ref > 0)
    assert np.max(np.abs(sr / ref - 1)) < 1e-5


@pytest.mark.parametrize("name", sorted(DISPLAYS))
def test_lmfr_shading_rate_matches_eq16(O, paper, name):
    """0.5 du/de of the oracle's LMFR map (Eq. (14)) equals the printed
    Eq. (16): 2 z^3 LW(e)."""
    W, H = DISPLAYS[name]
    w, h = O.lmfr_dims(W, H, paper["lmfr_delta"]["value"])
    p = O.film_pitch(W, H)
    g = (0.45 * W, 0.4 * H)
    lnL = O.lmfr_L(W, H, g[0], g[1])
    alpha = float(paper["lmfr_alpha"]["value"])
    e = np.linspace(1.0, 45.0, 30)

    def fwd(xy):
        return O.lmfr_forward(W, H, g[0], g[1], w, h, alpha, xy)[0]

    sr = _numeric_sr(O, W, H, p, g, w, h, e, fwd)
    z = np.log(np.tan(np.radians(e)) / p[1]) / lnL
    ref = 2 * z ** 3 * _lw(e, w, lnL)
    assert np.max(np.abs(sr / ref - 1)) < 1e-5


def test_lafr_pieces_meet_at_the_foveal_boundary(O, paper):
    """Eq. (15): both pieces give U_ef at Z_ef = z(4.89 deg); the point at
    4.89 deg maps to U_ef w; the farthest corner maps to w (z = 1, Za = -1);
    a point within one pixel of the gaze maps to 0."""
    lp = paper["lafr_parameters"]
    W, H = 3840, 2160
    w, h = O.lmfr_dims(W, H, 1.8)
    p = O.film_pitch(W, H)
    g = (1500.0, 900.0)
    c = O.lafr_consts(W, H, p, g[0], g[1])
    lnL, Zef, Fa, Uef = c
    assert abs(Zef - math.log(math.tan(math.radians(lp["foveal_boundary_deg"])) / p[1]) / lnL) < 1e-15
    below, above = O.lafr_u(c, [Zef, Zef * (1 + 1e-12)])
    assert abs(below - Uef) < 1e-14 and abs(above - Uef) < 1e-9
    r_ef = math.tan(math.radians(lp["foveal_boundary_deg"])) / p[1]
    u, v = O.lafr_forward(W, H, p, g[0], g[1], w, h, [[g[0], g[1] + r_ef], [W, H], [g[0] + 0.5, g[1]],
                                                      [g[0] - 50.0, g[1]]])
    assert abs(u[0] - Uef * w) < 1e-9 * w
    assert abs(u[1] - w) < 1e-9 * w
    assert u[2] == 0.0
    assert abs(v[3] - 0.5 * h) < 1e-9


def test_lafr_map_is_increasing_and_spans_the_buffer(O, paper):
    """u(z) rises from 0 to 1 over z in [0, 1], for the paper's own and its
    retinal-resolution parameters."""
    lp = paper["lafr_parameters"]
    W, H = 11520, 6480
    p = O.film_pitch(W, H)
    z = np.linspace(0.0, 1.0, 20001)
    for prm in (lp["original"], lp["tuned_retinal"]):
        c = O.lafr_consts(W, H, p, 0.5 * W, 0.5 * H, O.LAFR_A, prm["alpha"])
        u = O.lafr_u(c, z, prm["beta"])
        assert u[0] == 0.0 and abs(u[-1] - 1.0) < 1e-12
        assert np.all(np.diff(u) > 0)


def test_lafr_inverse_inverts_forward(O, paper):
    """The texel-to-screen direction (inverse of Eq. (15)) undoes the forward
    map on both pieces, for beta = 0.7 and the tuned beta = 0.9."""
    lp = paper["lafr_parameters"]
    W, H = 7680, 4320
    p = O.film_pitch(W, H)
    for prm in (lp["original"], lp["tuned_retinal"]):
        c = O.lafr_consts(W, H, p, 2000.0, 3000.0, O.LAFR_A, prm["alpha"])
        t = np.linspace(1e-4, 1 - 1e-4, 4001)
        z = O.lafr_z(c, t, prm["beta"])
        assert np.all(np.diff(z) > 0)
        assert np.max(np.abs(O.lafr_u(c, z, prm["beta"]) - t)) < 1e-12


def test_lafr_texel_rays_round_trip(O):
    """Texel (i, j)'s ray passes through the screen point that the forward
    map sends to (i + 1/2, j + 1/2)."""
    W, H = 1920, 1080
    w, h = O.lmfr_dims(W, H, 2.2)
    gx, gy = 700.25, 400.5
    p = O.film_pitch(W, H, 100.0, 100.0)
    cam = np.array([0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1], np.float32)
    rng = np.random.default_rng(16)
    idx = rng.integers(0, w * h, 4000)
    _, d = O.lafr_rays(W, H, p, gx, gy, w, h, idx, cam)
    X = d[:, 0].astype(float) / d[:, 2]
    Y = -d[:, 1].astype(float) / d[:, 2]
    xy = np.stack([X / p[0] + W / 2, Y / p[1] + H / 2], 1)
    u, v = O.lafr_forward(W, H, p, gx, gy, w, h, xy)
    i, j = idx // h, idx % h
    r = np.hypot(xy[:, 0] - gx, xy[:, 1] - gy)
    ok = r > 2.0
    assert np.max(np.abs(u[ok] - (i[ok] + 0.5))) < 2e-2
    dv = (v - (j + 0.5) + h / 2) % h - h / 2
    assert np.max(np.abs(dv[ok] * r[ok] / h)) < 1e-2


def test_lafr_kernel_defined_at_the_papers_settings(O, paper):
    """Z_ef and Fa lie in (0, 1) at every Table 1 resolution, gaze at the
    centre or a corner, for LaFR's own parameters; and at the retinal
    resolution for the tuned ones."""
    lp = paper["lafr_parameters"]
    t1 = paper["table1_rays_per_eye"]["resolutions"]
    for W, H in t1.values():
        p = O.film_pitch(W, H)
        for g in ((0.5 * W, 0.5 * H), (0.0, 0.0), (W, H)):
            lnL, Zef, Fa, Uef = O.lafr_consts(W, H, p, g[0], g[1], O.LAFR_A, lp["original"]["alpha"])
            assert 0 < Zef < 1 and 0 < Fa < 1 and 0 < Uef < Zef
    W, H = t1["Retinal"]
    O.lafr_consts(W, H, O.film_pitch(W, H), 0.5 * W, 0.5 * H, O.LAFR_A, lp["tuned_retinal"]["alpha"])


def test_lafr_shading_rate_jumps_at_the_foveal_boundary(O, paper):
    """Sec. 4.2: LaFR truncates its shading rate at the foveal boundary, with
    a blurrier image inside it; the radial rate just inside 4.89 deg is below
    the rate just outside."""
    lp = paper["lafr_parameters"]
    W, H = 2560, 1440
    w, h = O.lmfr_dims(W, H, 1.8)
    p = O.film_pitch(W, H)
    g = (0.5 * W, 0.5 * H)

    def fwd(xy):
        return O.lafr_forward(W, H, p, g[0], g[1], w, h, xy)[0]

    eb = lp["foveal_boundary_deg"]
    inside, outside = _numeric_sr(O, W, H, p, g, w, h, np.array([eb - 0.01, eb + 0.01]), fwd, de=1e-3)
    assert inside < 0.5 * outside


def test_lafr_reconstruct_samples_texel_centres(O):
    """A pixel centre that maps exactly onto a texel centre returns that
    texel; the buffer wraps in angle."""
    W, H = 640, 360
    w, h = O.lmfr_dims(W, H, 1.8)
    p = O.film_pitch(W, H)
    gx, gy = 320.5, 180.5     # gaze on a pixel centre
    rng = np.random.default_rng(3)
    lp = rng.random((w * h, 4), dtype=np.float32)
    # pixel straight right of the gaze: polar angle 0, between rows h-1 and 0
    pix = np.array([180 * W + 500], np.int64)
    out, _ = O.lafr_reconstruct(W, H, p, gx, gy, w, h, lp, pix)
    u, v = O.lafr_forward(W, H, p, gx, gy, w, h, [[500.5, 180.5]])
    ac = u[0] - 0.5
    i0 = int(math.floor(ac))
    wc = ac - i0
    ref = 0.5 * ((1 - wc) * (lp[i0 * h + h - 1] + lp[i0 * h]) + wc * (lp[(i0 + 1) * h + h - 1] + lp[(i0 + 1) * h]))
    assert abs(v[0]) < 1e-12
    assert np.max(np.abs(out[0] - ref)) < 1e-6
