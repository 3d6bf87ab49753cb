"""Pins for the oracle's ray casting, shading and reconstruction.

Closed forms, brute force on tiny inputs, watertightness on closed meshes and
invariants of the inverse map (Sec. 3.2.3, Sec. 6.1).
"""
import math

import numpy as np
import pytest

from paper_2503_23410_amd import inputs as I


# ------------------------------------------------------- ray / triangle ---

def test_watertight_closed_forms(O):
    """Axis-aligned triangle z = 2 spanning x, y in [0, 1]: hits at t = 2
    inside (both windings), misses outside, misses behind the origin."""
    tri = np.array([0, 0, 2, 1, 0, 2, 0, 1, 2], np.float32)
    tri_rev = np.array([0, 0, 2, 0, 1, 2, 1, 0, 2], np.float32)
    org = np.zeros((5, 3), np.float32)
    d = np.array([[0.25, 0.25, 1.0], [0.125, 0.125, 1.0], [0.6, 0.6, 1.0], [0.25, 0.25, -1.0], [0.2, 0.2, 0.0]],
                 np.float32)
    for t9 in (tri, tri_rev):
        hit, t, m = O.watertight_many(org, d, np.tile(t9, (5, 1)))
        assert list(hit) == [True, True, False, False, False]
        assert t[0] == np.float32(2.0) and t[1] == np.float32(2.0)
    # barycentric margin: hit point (0.5, 0.25) has weights (0.25, 0.5, 0.25)
    hit, t, m = O.watertight_many(org[:1], np.array([[0.25, 0.125, 1.0]], np.float32), tri[None, :])
    assert hit[0] and abs(m[0] - 0.25) < 1e-6
    # a miss by 0.01 outside the edge x + y = 1: margin is the outside weight
    hit, t, m = O.watertight_many(org[:1], np.array([[0.255, 0.25, 1.0]], np.float32), tri[None, :])
    assert not hit[0] and abs(m[0] - 0.01 / 1.02) < 1e-5


def test_watertight_edges_and_vertices_count_as_hits(O):
    """Rays through a shared edge hit at least one of the two triangles, and
    rays through an exact vertex hit."""
    # unit square at z = 1 split along its diagonal
    a = np.array([[0, 0, 1], [1, 0, 1], [1, 1, 1]], np.float32).reshape(-1)
    b = np.array([[0, 0, 1], [1, 1, 1], [0, 1, 1]], np.float32).reshape(-1)
    s = np.linspace(0.0, 1.0, 257, dtype=np.float32)
    d = np.stack([s, s, np.ones_like(s)], 1)            # exactly on the diagonal
    org = np.zeros_like(d)
    ha, _, _ = O.watertight_many(org, d, np.tile(a, (s.size, 1)))
    hb, _, _ = O.watertight_many(org, d, np.tile(b, (s.size, 1)))
    assert np.all(ha | hb)


def test_icosphere_is_watertight_from_inside(O):
    """Closed mesh: rays from the centre through every vertex, every edge
    midpoint and random directions never miss (Woop et al.'s guarantee)."""
    v, f = I.icosphere(3)
    v = (v * 0.7 + np.array([0.1, -0.2, 0.3])).astype(np.float32)
    sc = O.Scene(v, f.astype(np.int32), use_bvh=False)
    c = np.array([0.1, -0.2, 0.3], np.float32)
    edges = set()
    for a, b, cc in f:
        for p, q in ((a, b), (b, cc), (cc, a)):
            edges.add((min(p, q), max(p, q)))
    mids = np.array([(v[p].astype(float) + v[q]) / 2 for p, q in edges])
    rng = np.random.default_rng(21)
    rnd = rng.normal(size=(3000, 3))
    targets = np.concatenate([v.astype(float), mids, c + rnd])
    d = (targets - c).astype(np.float32)
    org = np.tile(c, (d.shape[0], 1))
    ids, t, fl = sc.closest(org, d)
    assert np.all(ids >= 0)
    occ, _ = sc.any(org, d)
    assert np.all(occ)


def test_closest_hit_tie_break_by_id(O):
    """Two coincident triangles: the smaller id wins (equal t)."""
    tri = np.array([[-1, -1, 1], [1, -1, 1], [0, 1, 1]], np.float32)
    v = np.concatenate([tri, tri])
    f = np.array([[0, 1, 2], [3, 5, 4]], np.int32)
    sc = O.Scene(v, f, use_bvh=False)
    ids, t, fl = sc.closest(np.zeros((1, 3), np.float32), np.array([[0.1, 0.0, 1.0]], np.float32))
    assert ids[0] == 0 and t[0] == np.float32(1.0) and fl[0] == 1   # exact tie is flagged


def test_bvh_equals_brute_force_soup(O):
    """Closest-hit ids and t from the oracle BVH equal brute force on the
    4,096-triangle soup for rays from several origins."""
    v, f = I.soup_scene()
    bf = O.Scene(v, f, use_bvh=False)
    bv = O.Scene(v, f, use_bvh=True)
    rng = np.random.default_rng(22)
    n = 6000
    org = np.concatenate([np.tile([0, 0, -3], (n // 2, 1)), rng.uniform(-1.5, 1.5, (n - n // 2, 3))])
    org = org.astype(np.float32)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    d[: n // 2, 2] = np.abs(d[: n // 2, 2]) + 0.5
    i1, t1, f1 = bf.closest(org, d)
    i2, t2, f2 = bv.closest(org, d)
    assert np.array_equal(i1, i2)
    assert np.array_equal(t1, t2)
    assert np.array_equal(f1, f2)
    o1, g1 = bf.any(org, d)
    o2, g2 = bv.any(org, d)
    assert np.array_equal(o1, o2)
    assert (ids_hit := (i1 >= 0)).mean() > 0.3
    assert np.array_equal(o1, ids_hit)   # any-hit agrees with closest-hit


def test_bvh_equals_brute_force_terrain_sample(O):
    """Same on a heightfield + icosphere scene (brute force over all
    triangles for a small ray sample)."""
    v, f = I.terrain_scene(64, 32, 16, seed=9)
    bf = O.Scene(v, f, use_bvh=False)
    bv = O.Scene(v, f, use_bvh=True)
    W, H = 320, 180
    p = O.film_pitch(W, H, 100.0, 100.0)
    rng = np.random.default_rng(23)
    pix = rng.integers(0, W * H, 1500)
    org, d = O.full_rays(W, H, p, pix, I.terrain_camera())
    i1, t1, _ = bf.closest(org, d)
    i2, t2, _ = bv.closest(org, d)
    assert np.array_equal(i1, i2) and np.array_equal(t1, t2)
    assert (i1 >= 0).mean() > 0.8


def test_heightfield_grid_has_no_cracks(O):
    """Rays aimed exactly at grid vertices and edge midpoints of a flat
    heightfield always hit (shared edges are watertight)."""
    v, f = I.terrain_scene(32, 16, 0, seed=5)
    v[:, 1] = -0.6                      # flatten: vertices become exact targets
    sc = O.Scene(v, f, use_bvh=True)
    eye = np.array([0.013, 0.5, -0.021], np.float32)
    tg = np.concatenate([v.astype(float), (v[f[:, 0]].astype(float) + v[f[:, 1]]) / 2])
    inside = (np.abs(tg[:, 0]) < 1.99) & (np.abs(tg[:, 2]) < 0.99)
    d = (tg[inside] - eye).astype(np.float32)
    ids, _, _ = sc.closest(np.tile(eye, (d.shape[0], 1)), d)
    assert np.all(ids >= 0)


# -------------------------------------------------------------- shading ---

def _quad_scene(z=2.0, size=50.0):
    v = np.array([[-size, -size, z], [size, -size, z], [size, size, z], [-size, size, z]], np.float32)
    f = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return v, f


def test_lambert_closed_form(O):
    """Single plane facing the camera: colour = albedo (ambient + L max(0,n.l)),
    n faced toward the viewer; misses take the background."""
    v, f = _quad_scene()
    sc = O.Scene(v, f, use_bvh=False)
    sh = O.shading_params(light_dir=(0.0, 0.6, -0.8))
    org = np.zeros((3, 3), np.float32)
    d = np.array([[0.1, 0.2, 1.0], [-0.3, 0.1, 1.0], [0.0, 0.0, -1.0]], np.float32)
    rgba, ids, fl = sc.shade(org, d, sh)
    alb = O.albedo(ids[:2])
    ndl = np.float32(0.8)                    # n = (0, 0, -1) faces the eye
    want = alb * (np.float32(0.1) + ndl)
    assert np.allclose(rgba[:2, :3], want, atol=1e-6)
    assert np.allclose(rgba[2], [0.05, 0.05, 0.08, 1.0])
    assert np.all(rgba[:, 3] == 1.0)


def test_shadow_ray_blocks_light(O):
    """An occluder between the plane and the light leaves ambient only;
    with shadows off the full Lambert term returns."""
    v, f = _quad_scene()
    occ = np.array([[-1, -1, 1.0], [1, -1, 1.0], [0, 1, 1.0]], np.float32)   # in front, toward the light
    v2 = np.concatenate([v, occ + np.array([0, 0, -0.5], np.float32)])
    f2 = np.concatenate([f, np.array([[4, 5, 6]], np.int32)])
    sc = O.Scene(v2, f2, use_bvh=True)
    # light toward -z: the shadow ray from the plane point (0, 0, 2) runs
    # back along -z and meets the occluder at z = 0.5; the primary ray from
    # (3, 0, -5) crosses z = 0.5 at x = 0.64, beside the occluder.
    sh = O.shading_params(light_dir=(0.0, 0.0, -1.0))
    org = np.array([[3.0, 0.0, -5.0]], np.float32)
    d = np.array([[-3.0, 0.0, 7.0]], np.float32)
    rgba, ids, _ = sc.shade(org, d, sh)
    assert ids[0] in (0, 1)
    alb = O.albedo(ids)
    assert np.allclose(rgba[0, :3], alb[0] * np.float32(0.1), atol=1e-6)
    rgba2, _, _ = sc.shade(org, d, O.shading_params(light_dir=(0.0, 0.0, -1.0), shadow=False))
    assert np.allclose(rgba2[0, :3], alb[0] * np.float32(1.1), atol=1e-6)


def test_albedo_hash_is_a_bijection_with_uniform_bytes(O):
    """The 32-bit hash behind the albedo is a permutation (no collisions on
    2^20 consecutive ids) with near-uniform bytes; albedo is in [0.2, 0.9]."""
    ids = np.arange(1 << 20, dtype=np.int32)
    a = O.albedo(ids)
    assert a.min() >= 0.2 - 1e-7 and a.max() <= 0.9 + 1e-6
    q = np.round((a - 0.2) / 0.7 * 255).astype(np.int64)
    key = q[:, 0] | (q[:, 1] << 8) | (q[:, 2] << 16)
    # 24 bits of a bijective 32-bit hash over 2^20 ids: collisions ~ Poisson
    assert len(np.unique(key)) > (1 << 20) * 0.96
    for ch in range(3):
        h = np.bincount(q[:, ch], minlength=256)
        assert h.min() > 0.85 * (1 << 20) / 256 and h.max() < 1.15 * (1 << 20) / 256


def test_path_mode_zero_bounces_equals_lambert(O):
    """Path-traced shading with no continuation ray reduces to the Lambert +
    shadow shading (same vertex term)."""
    v, f = I.soup_scene()
    sc = O.Scene(v, f, use_bvh=True)
    W, H = 64, 36
    p = O.film_pitch(W, H, 100.0, 100.0)
    pix = np.arange(W * H)
    org, d = O.full_rays(W, H, p, pix, I.soup_camera())
    sh = O.shading_params()
    a, ia, _ = sc.shade(org, d, sh)
    b, ib, _ = sc.shade_path(org, d, pix, sh, seed=7, frame=0, view=0, bounces=0)
    assert np.array_equal(ia, ib)
    assert np.allclose(a, b, atol=1e-6)


def test_path_mode_open_plane_closed_form(O):
    """An upward plane under an open sky: the first bounce always escapes, so
    L = a (ambient + n.l) + a * background exactly (bounces >= 1)."""
    v = np.array([[-50, 0, -50], [50, 0, -50], [50, 0, 50], [-50, 0, 50]], np.float32)
    f = np.array([[0, 2, 1], [0, 3, 2]], np.int32)
    sc = O.Scene(v, f, use_bvh=False)
    sh = O.shading_params(light_dir=(0.0, 1.0, 0.0), background=(0.3, 0.2, 0.1))
    n = 200
    rng = np.random.default_rng(24)
    org = np.tile(np.array([0, 1.0, 0], np.float32), (n, 1))
    d = np.concatenate([rng.uniform(-0.5, 0.5, (n, 1)), -np.ones((n, 1)), rng.uniform(-0.5, 0.5, (n, 1))], 1)
    d = d.astype(np.float32)
    rgba, ids, _ = sc.shade_path(org, d, np.arange(n), sh, seed=3, frame=1, view=2, bounces=2)
    alb = O.albedo(ids)
    want = alb * (np.float32(0.1) + np.float32(1.0)) + alb * np.array([0.3, 0.2, 0.1], np.float32)
    assert np.allclose(rgba[:, :3], want, atol=1e-5)


def test_cosine_sampling_statistics(O):
    """Cosine-weighted hemisphere sampling: E[cos] = 2/3, E[cos^2] = 1/2.
    Measured through the path mode on a plane under a sky whose only light
    is the background, seen from the continuation ray: with an overhead
    blocker plane at height h the escape fraction is known in closed form.
    Here: a blocker covering the full upper half-space except a cone of
    half-angle 60 degrees about +y; the escape probability under cosine
    sampling is sin^2(60) = 0.75."""
    # ground plane y = 0, a large annulus-like blocker is hard to build with
    # triangles; instead use a square hole: roof at y = 1 with a 2 x 2 hole
    # centred above the ray footprint.  Escape probability for cosine
    # sampling through a square hole of half-width a at height h from the
    # centre: computed by numerical integration below.
    roof = []
    big, a = 100.0, 1.0
    for x0, x1, z0, z1 in ((-big, -a, -big, big), (a, big, -big, big), (-a, a, -big, -a), (-a, a, a, big)):
        roof.append([[x0, 1, z0], [x1, 1, z0], [x1, 1, z1], [x0, 1, z1]])
    verts = [[-50, 0, -50], [50, 0, -50], [50, 0, 50], [-50, 0, 50]]
    faces = [[0, 2, 1], [0, 3, 2]]
    for q in roof:
        b = len(verts)
        verts += q
        faces += [[b, b + 1, b + 2], [b, b + 2, b + 3]]
    sc = O.Scene(np.array(verts, np.float32), np.array(faces, np.int32), use_bvh=True)
    sh = O.shading_params(light_dir=(0.0, 1.0, 0.0), light_rgb=(0, 0, 0), ambient=(0, 0, 0),
                          background=(1.0, 1.0, 1.0))
    n = 40000
    org = np.tile(np.array([0, 0.5, 0], np.float32), (n, 1))
    d = np.tile(np.array([0, -1.0, 0], np.float32), (n, 1))
    rgba, ids, _ = sc.shade_path(org, d, np.arange(n), sh, seed=11, frame=0, view=0, bounces=1)
    alb = O.albedo(ids)
    frac = rgba[:, 0] / alb[:, 0]
    # escape probability through the square hole [-1,1]^2 at height 1 for a
    # cosine-weighted lobe about +y: (1/pi) * integral over the hole of
    # cos^2 / dist^2 ... = (1/pi) * int int h^2 / (x^2+z^2+h^2)^2 dx dz
    g = np.linspace(-1, 1, 801)
    X, Z = np.meshgrid(g, g)
    integrand = 1.0 / (X ** 2 + Z ** 2 + 1.0) ** 2
    p_escape = np.trapezoid(np.trapezoid(integrand, g, axis=1), g) / np.pi
    assert abs(frac.mean() - p_escape) < 4 * math.sqrt(p_escape * (1 - p_escape) / n)


def test_rng_is_uniform_and_keyed(O):
    """Counter-based uniform numbers in [0, 1) with 24-bit resolution; every
    key word changes the value."""
    xs = np.array([O.rng01(5, 0, 0, t, 0) for t in range(20000)])
    assert xs.min() >= 0 and xs.max() < 1
    assert abs(xs.mean() - 0.5) < 0.01 and abs(xs.var() - 1 / 12) < 0.005
    base = O.rng01(5, 1, 2, 3, 4)
    for k in range(5):
        key = [5, 1, 2, 3, 4]
        key[k] += 1
        assert O.rng01(*key) != base
    assert np.all(np.abs(xs * 16777216 - np.round(xs * 16777216)) < 1e-6)


# ------------------------------------------------------- reconstruction ---

def _pix_all(W, H):
    return np.arange(W * H, dtype=np.int64)


def test_reconstruct_constant_is_exact(O, layout):
    """A constant LP buffer reconstructs to exactly that constant everywhere,
    for a central and a far off-centre gaze (e > 60 degrees clamps)."""
    W, H = 320, 180
    p = O.film_pitch(W, H, 100.0, 100.0)
    lp = np.tile(np.array([0.25, 0.5, 0.75, 1.0], np.float32), (layout.n_texels, 1))
    for gaze in ((160.0, 90.0), (0.0, 0.0), (319.0, 2.0)):
        G = O.gaze_film(W, H, p, *gaze)
        out, _ = O.vafr_reconstruct(layout, lp, W, H, p, G, _pix_all(W, H))
        assert np.all(out == lp[0])


def test_reconstruct_linear_in_column_index(O, layout):
    """LP = a + b i (constant along each column): the column filter is linear
    in u, so the image equals a + b (clamp(u, 1/2, N_c - 1/2) - 1/2) with u
    from the forward map (Eq. (5))."""
    W, H = 400, 300
    p = O.film_pitch(W, H, 100.0, 100.0)
    G = O.gaze_film(W, H, p, 123.0, 77.0)
    col = np.repeat(np.arange(layout.n_cols), layout.n_rows).astype(np.float64)
    lp = np.zeros((layout.n_texels, 4), np.float32)
    lp[:, 0] = (0.001 * col).astype(np.float32)
    out, _ = O.vafr_reconstruct(layout, lp, W, H, p, G, _pix_all(W, H))
    xs = np.stack(np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5), -1).reshape(-1, 2)
    u, _, _, _ = O.vafr_forward(layout.acuity, W, H, p, G, xs)
    want = 0.001 * (np.clip(u, 0.5, layout.n_cols - 0.5) - 0.5)
    assert np.max(np.abs(out[:, 0] - want)) < 2e-6


def test_reconstruct_recovers_screen_position(O, layout):
    """End-to-end consistency of the layout tables and the inverse map: store
    in every texel the film position of its own ray (G + dxy, Sec. 6.1);
    the reconstructed image is then the film position of each pixel, up to
    the interpolation error of the LP grid (a sign or orientation error
    would mirror it)."""
    W, H = 480, 270
    p = O.film_pitch(W, H, 100.0, 100.0)
    G = O.gaze_film(W, H, p, 300.0, 100.0)
    lp = np.zeros((layout.n_texels, 4), np.float32)
    lp[:, 0] = (G[0] + layout.dxy[0::2].astype(float)).astype(np.float32)
    lp[:, 1] = (G[1] + layout.dxy[1::2].astype(float)).astype(np.float32)
    out, _ = O.vafr_reconstruct(layout, lp, W, H, p, G, _pix_all(W, H))
    x = (np.arange(W * H) % W + 0.5 - W / 2) * p[0]
    y = (np.arange(W * H) // W + 0.5 - H / 2) * p[1]
    rho = np.hypot(x - G[0], y - G[1])
    e = np.degrees(np.arctan(rho))
    ok = e < 59.0
    # interpolation error of a position on a polar grid of spacing s: O(s^2/r)
    err = np.hypot(out[ok, 0] - x[ok], out[ok, 1] - y[ok])
    assert np.median(err / p.min()) < 0.1
    assert np.max(err / p.min()) < 2.0


def test_reconstruct_wraps_at_theta_zero(O, layout):
    """Pixels just above and below the +x ray from the gaze read the same rows
    across the 0/360 seam: a smooth LP in theta gives a continuous image."""
    W, H = 801, 601
    p = O.film_pitch(W, H, 100.0, 100.0)
    gaze = (400.5, 300.5)
    G = O.gaze_film(W, H, p, *gaze)
    col = np.repeat(np.arange(layout.n_cols), layout.n_rows)
    row = np.arange(layout.n_texels) - layout.col_off[col]
    th = 2 * np.pi * (row + 0.5) / layout.n_rows[col]
    lp = np.zeros((layout.n_texels, 4), np.float32)
    lp[:, 0] = np.cos(th)
    # pixel rows 300 and 301 straddle the gaze's horizontal line (y = 300.5)
    xs = np.arange(420, 800)
    above = 300 * W + xs
    below = 301 * W + xs
    a, _ = O.vafr_reconstruct(layout, lp, W, H, p, G, above)
    b, _ = O.vafr_reconstruct(layout, lp, W, H, p, G, below)
    assert np.max(np.abs(a[:, 0] - b[:, 0])) < 0.02
    assert np.all(a[:, 0] > 0.9)


def test_reconstruct_flags_propagate(O, layout):
    """A pixel is flagged iff it reads a flagged texel."""
    W, H = 64, 64
    p = O.film_pitch(W, H, 100.0, 100.0)
    G = O.gaze_film(W, H, p, 32.0, 32.0)
    lp = np.ones((layout.n_texels, 4), np.float32)
    tf = np.zeros(layout.n_texels, np.uint8)
    _, pf = O.vafr_reconstruct(layout, lp, W, H, p, G, _pix_all(W, H), tf)
    assert not pf.any()
    tf[:] = 1
    _, pf = O.vafr_reconstruct(layout, lp, W, H, p, G, _pix_all(W, H), tf)
    assert pf.all()


def test_lmfr_reconstruct_constant_and_linear(O):
    """LMFR inverse map: constant in -> constant out; LP = a + b i -> image
    a + b (clamp(u) - 1/2) with u from Eq. (1)/(14)."""
    W, H = 360, 200
    w, h = O.lmfr_dims(W, H, 1.8)
    gx, gy = 100.0, 150.0
    lp = np.tile(np.array([0.1, 0.2, 0.3, 1.0], np.float32), (w * h, 1))
    out, _ = O.lmfr_reconstruct(W, H, gx, gy, w, h, 4.0, lp, _pix_all(W, H))
    assert np.all(out == lp[0])
    i = np.arange(w * h) // h
    lp2 = np.zeros((w * h, 4), np.float32)
    lp2[:, 0] = 0.01 * i
    out, _ = O.lmfr_reconstruct(W, H, gx, gy, w, h, 4.0, lp2, _pix_all(W, H))
    xs = np.stack(np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5), -1).reshape(-1, 2)
    u, _ = O.lmfr_forward(W, H, gx, gy, w, h, 4.0, xs)
    want = 0.01 * (np.clip(u, 0.5, w - 0.5) - 0.5)
    assert np.max(np.abs(out[:, 0] - want)) < 1e-5


# ------------------------------------------------- near-tie flag branches ---
#
# Flagged rays are left out of every exact id comparison, so each branch of
# the flag must fire where a near tie really exists and stay quiet on clean
# hits and misses; an over-eager flag would silently widen every parity test.
# The right triangle (0,0), (1,0), (0,1) in the plane z = zp, seen from the
# origin: the ray through film point (x, y) meets it at (x zp, y zp), whose
# barycentric weights are (1 - zp(x + y), zp x, zp y).

def _tri_at(zp, dx=0.0):
    return np.array([[dx, 0, zp], [dx + 1, 0, zp], [dx, 1, zp]], np.float32)


def _scene_of(O, *tris):
    v = np.concatenate(tris).astype(np.float32)
    f = np.arange(v.shape[0], dtype=np.int32).reshape(-1, 3)
    return O.Scene(v, f, use_bvh=False), O.Scene(v, f, use_bvh=True)


def _closest_both(O, scenes, d):
    out = []
    for sc in scenes:
        ids, t, fl = sc.closest(np.zeros((len(d), 3), np.float32), np.asarray(d, np.float32))
        out.append((ids, t, fl))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][2], out[1][2])
    return out[0]


# a film point 5e-7 inside the hypotenuse x + y = 1 of the triangle at z = 1,
# one 5e-7 outside it, and a clean interior point
_NEAR_IN = (0.25, 0.75 - 5e-7, 1.0)
_NEAR_OUT = (0.25, 0.75 + 5e-7, 1.0)
_CLEAN = (0.25, 0.25, 1.0)


def test_flag_setup_margins(O):
    """The film points above are what their names say under the watertight
    test itself: a hit with margin below 1e-6, a miss with margin below
    1e-6, and a hit with margin 0.25."""
    tri = _tri_at(1.0).reshape(1, 9)
    hit, t, m = O.watertight_many(np.zeros((3, 3), np.float32), np.array([_NEAR_IN, _NEAR_OUT, _CLEAN],
                                                                          np.float32), np.tile(tri, (3, 1)))
    assert list(hit) == [True, False, True]
    assert 0 < m[0] < 1e-6 and 0 < m[1] < 1e-6 and abs(m[2] - 0.25) < 1e-6


def test_flag_winner_near_edge(O):
    """Branch 1: the winner's smallest barycentric weight is below 1e-6."""
    sc = _scene_of(O, _tri_at(1.0))
    ids, t, fl = _closest_both(O, sc, [_NEAR_IN, _CLEAN])
    assert list(ids) == [0, 0]
    assert list(fl) == [1, 0]


def test_flag_runner_up_within_relative_t(O):
    """Branch 2: a second hit lies within relative 1e-6 of the winner's t;
    a second hit 1e-4 behind does not flag."""
    z2_near = np.nextafter(np.float32(1.0), np.float32(2.0), dtype=np.float32) \
        + np.float32(2 ** -23)                           # 1 + 2^-22: relative gap 2.4e-7
    for z2, want in ((z2_near, 1), (np.float32(1.0001), 0)):
        sc = _scene_of(O, _tri_at(1.0), _tri_at(float(z2)))
        ids, t, fl = _closest_both(O, sc, [_CLEAN])
        assert ids[0] == 0 and t[0] == np.float32(1.0)
        assert fl[0] == want, (z2, fl[0])
    # the runner-up found first (nearer triangle stored second) flags too
    sc = _scene_of(O, _tri_at(float(z2_near)), _tri_at(1.0))
    ids, t, fl = _closest_both(O, sc, [_CLEAN])
    assert ids[0] == 1 and fl[0] == 1


def test_flag_near_miss_in_front_of_winner(O):
    """Branch 3: a triangle in front of the winner missed by less than 1e-6
    flags the ray; the same near miss behind the winner, or a clear miss in
    front, does not."""
    # winner: a large triangle at z = 2 containing the whole ray bundle
    big = np.array([[-10, -10, 2], [10, -10, 2], [0, 10, 2]], np.float32)
    for zp, d, want in ((1.0, _NEAR_OUT, 1), (1.0, (0.25, 0.76, 1.0), 0), (3.0, (0.25 / 3, (0.75 + 5e-7) / 3, 1.0),
                                                                             0)):
        sc = _scene_of(O, big, _tri_at(zp))
        hit, _, m = O.watertight_many(np.zeros((1, 3), np.float32), np.array([d], np.float32),
                                      _tri_at(zp).reshape(1, 9))
        ids, t, fl = _closest_both(O, sc, [d])
        assert not hit[0] and ids[0] == 0
        assert fl[0] == want, (zp, d, m[0], fl[0])


def test_flag_near_miss_on_a_missing_ray(O):
    """Branch 3 on a ray that hits nothing: a near miss anywhere in front
    flags it; a clear miss does not."""
    sc = _scene_of(O, _tri_at(1.0))
    ids, t, fl = _closest_both(O, sc, [_NEAR_OUT, (0.25, 0.8, 1.0), (0.25, 0.75 + 5e-7, -1.0)])
    assert list(ids) == [-1, -1, -1]
    assert list(fl) == [1, 0, 0]          # the last one points away: t < 0


def test_flag_shadow_ray_near_edge_only(O):
    """Any-hit (shadow) rays: only near-edge candidates flag (whether the
    test calls them hits or misses); a robust hit or a clean miss does
    not, and a robust hit outweighs a near-edge one."""
    z = np.zeros((1, 3), np.float32)
    cases = [((_tri_at(1.0),), _NEAR_IN, True, 1), ((_tri_at(1.0),), _NEAR_OUT, False, 1),
             ((_tri_at(1.0),), _CLEAN, True, 0), ((_tri_at(1.0),), (0.25, 0.8, 1.0), False, 0),
             ((_tri_at(1.0), np.array([[-9, -9, 3], [9, -9, 3], [0, 9, 3]], np.float32)), _NEAR_OUT, True, 0)]
    for tris, d, occ_want, fl_want in cases:
        for sc in _scene_of(O, *tris):
            occ, fl = sc.any(z, np.array([d], np.float32))
            assert occ[0] == occ_want and fl[0] == fl_want, (d, occ[0], fl[0])


def test_flag_shadow_branch_reaches_the_shaded_ray(O):
    """A primary ray with a clean closest hit whose shadow ray only grazes
    an occluder's edge is flagged by the shading step; moved 1e-2 away from
    the edge it is not.  The primary ray comes in at 45 degrees so that it
    passes nowhere near the occluder itself."""
    ground = np.array([[-4, 0, -4], [4, 0, -4], [0, 0, 4]], np.float32)
    org = np.array([[-0.625, 1.0, 0.125]], np.float32)
    d = np.array([[1.0, -1.0, 0.0]], np.float32)           # hits (0.375, 0, 0.125) at t = 1
    sh = O.shading_params(light_dir=(0.0, 1.0, 0.0))
    for gap, want in ((5e-7, 1), (1e-2, 0)):
        x0 = np.float32(0.375) + np.float32(gap)
        occl = np.array([[x0, 0.5, -1.0], [x0, 0.5, 1.0], [x0 + 2.0, 0.5, 0.0]], np.float32)
        v = np.concatenate([ground, occl])
        f = np.arange(6, dtype=np.int32).reshape(2, 3)
        for sc in (O.Scene(v, f, use_bvh=False), O.Scene(v, f, use_bvh=True)):
            ids, t, cfl = sc.closest(org, d)
            assert ids[0] == 0 and t[0] == np.float32(1.0) and cfl[0] == 0
            rgba, sid, sfl = sc.shade(org, d, sh)
            assert sid[0] == 0 and sfl[0] == want, (gap, sfl[0])
            # the shadow ray misses the occluder in both cases: full light
            alb = O.albedo([0])[0]
            assert np.allclose(rgba[0, :3], alb * (0.1 + 1.0), atol=1e-6)


def test_reconstruction_taps_are_its_footprint(O, layout):
    """vafr_taps lists the texels each pixel reads: an LP buffer that is 1
    at one texel and 0 elsewhere reconstructs to non-zero values only at
    pixels whose taps hold that texel, and a flag on that texel reaches
    exactly the pixels whose taps hold it."""
    W, H = 320, 180
    p = O.film_pitch(W, H, 100.0, 100.0)
    G = O.gaze_film(W, H, p, 150.3, 70.9)
    pix = np.arange(W * H)
    taps = O.vafr_taps(layout, W, H, p, G, pix)
    assert taps.shape == (W * H, 4) and taps.min() >= 0 and taps.max() < layout.n_texels
    rng = np.random.default_rng(1)
    for k in rng.choice(np.unique(taps), 12, replace=False):
        lp = np.zeros((layout.n_texels, 4), np.float32)
        lp[k] = 1.0
        fl = np.zeros(layout.n_texels, np.uint8)
        fl[k] = 1
        img, pf = O.vafr_reconstruct(layout, lp, W, H, p, G, pix, fl)
        has = (taps == k).any(axis=1)
        assert not ((img[:, 0] != 0) & ~has).any()
        assert np.array_equal(pf, has)
