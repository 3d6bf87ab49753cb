"""Pins for the oracle's binocular reprojection by forward grid warping
(Sec. 5.1): the zipper triangulation tiles every band of the LP grid, one
camera gives back the left buffer, depth is interpolated perspective-correctly
(exact on a plane), depth jumps are not bridged, and the baseline shifts
points by b / z on the film."""
import ctypes as C

import numpy as np
import pytest

from paper_2503_23410_amd import inputs as I


def _tris(O, n_rows):
    n_rows = np.asarray(n_rows, np.int32)
    col_off = np.concatenate([[0], np.cumsum(n_rows)]).astype(np.int64)
    lib = O.lib()
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    m = int(lib.or_warp_triangles(len(n_rows), P(n_rows), P(col_off), None, None))
    v = np.empty((m, 3), np.int64)
    ids = np.empty(m, np.int64)
    lib.or_warp_triangles(len(n_rows), P(n_rows), P(col_off), P(v), P(ids))
    return n_rows, col_off, v, ids


@pytest.mark.parametrize("rows", [[4, 10, 16, 22], [3, 3, 7, 2, 9], [1, 5, 5, 1], [6, 4]])
def test_zipper_tiles_each_band_exactly_once(O, rows):
    """In (column + 1/2, angle) coordinates every point of a band between
    two columns lies in exactly one of the band's triangles (brute force)."""
    n_rows, col_off, v, ids = _tris(O, rows)
    n = int(col_off[-1])
    col = np.repeat(np.arange(len(n_rows)), n_rows)
    row = np.arange(n) - col_off[col]
    pu = col + 0.5
    pa = (row + 0.5) / n_rows[col]
    assert len(ids) == 2 * n - n_rows[0] - n_rows[-1]
    assert np.unique(ids).size == len(ids)
    x = v[:, 1]
    # ids: 2x + 1 when x is the band's inner column, 2x otherwise
    inner = col[v[:, 2]] > col[x]
    assert np.array_equal(ids, 2 * x + inner)
    rng = np.random.default_rng(7)
    for s in range(len(n_rows) - 1):
        band = col[x] + np.where(inner, 0, -1) == s
        tv = v[band]
        # unwrapped angles: the previous texel of x's column comes strictly
        # before x, the other column's texel before x in the merged order
        # (on equal angles the inner column first)
        ax = pa[tv[:, 1]]
        A = pa[tv].copy()
        A[:, 0] -= A[:, 0] >= ax
        later = (A[:, 2] > ax) | ((A[:, 2] == ax) & (col[tv[:, 2]] > col[tv[:, 1]]))
        A[:, 2] -= later
        U = pu[tv]
        pts_u = rng.uniform(s + 0.5, s + 1.5, 4000)
        pts_a = rng.uniform(0.0, 1.0, 4000)
        hits = np.zeros(pts_u.size, int)
        for shift in (-1.0, 0.0, 1.0):
            qu, qa = pts_u[:, None], pts_a[:, None] + shift
            def edge(i, j):
                return (U[:, j] - U[:, i])[None] * (qa - A[:, i][None]) - (A[:, j] - A[:, i])[None] * (qu - U[:, i][None])
            e0, e1, e2 = edge(1, 2), edge(2, 0), edge(0, 1)
            inside = ((e0 > 0) & (e1 > 0) & (e2 > 0)) | ((e0 < 0) & (e1 < 0) & (e2 < 0))
            hits += inside.sum(axis=1)
        assert np.all(hits == 1), (s, np.bincount(hits))


def test_same_camera_gives_back_the_left_buffer(O, layout):
    v, f = I.make_scene("terrain1m")
    sc = O.Scene(v, f)
    cam = I.terrain_camera()
    left, right, tri, fl, rid = O.rep_lp(sc, layout, 1920, 1080, I.FOV, (900.0, 500.0), cam, cam,
                                         O.shading_params())
    org, d = O.vafr_rays(layout, np.arange(layout.n_texels),
                         O.gaze_film(1920, 1080, O.film_pitch(1920, 1080, *I.FOV), 900.0, 500.0), cam)
    lid = sc.closest(org, d)[0]
    cov = (tri >= 0) & ~fl
    assert cov.mean() > 0.9 * (lid >= 0).mean()
    assert np.array_equal(rid[cov], lid[cov])
    # a texel's own point projects back onto its sample point up to FP32
    # rounding of the film coordinates (about 1e-3 of a foveal cell), so
    # its neighbours keep weights of that order
    assert np.abs(right[cov] - left[cov]).max() < 1e-3


def _plane_scene(y=-1.0, half=200.0):
    # one large triangle of the ground plane y = const
    vv = np.array([[-half, y, -half], [3 * half, y, -half], [-half, y, 3 * half]], np.float32)
    return vv, np.array([[0, 1, 2]], np.int32)


def test_depth_is_perspective_correct_on_a_plane(O, layout):
    """A ground plane seen at grazing angles: the warped depth equals the
    right eye's own ray-cast depth (1/z is linear on the film, z is not)."""
    vv, ff = _plane_scene()
    sc = O.Scene(vv, ff)
    cl, cr = I.binocular_cameras()
    cl = cl.copy(); cr = cr.copy()
    cl[:3] = (0.0, 0.0, -0.032); cr[:3] = (0.0, 0.0, 0.032)
    W, H, gz = 1920, 1080, (960.0, 540.0)
    depth = np.zeros(layout.n_texels, np.float32)
    left, right, tri, fl, rid = O.rep_lp(sc, layout, W, H, I.FOV, gz, cl, cr, O.shading_params(), depth=depth)
    G = O.gaze_film(W, H, O.film_pitch(W, H, *I.FOV), *gz)
    org, d = O.vafr_rays(layout, np.arange(layout.n_texels), G, cr)
    ids, t, _ = sc.closest(org, d)
    cov = (tri >= 0) & (ids >= 0)
    assert cov.sum() > 0.9 * (ids >= 0).sum()
    z_ray = t[cov].astype(np.float64) * (d[cov].astype(np.float64) @ cr[9:12].astype(np.float64))
    # FP32 film coordinates of the vertices limit the agreement near the
    # horizon to about 5e-5; interpolating z instead of 1/z errs up to 1e-3
    rel = np.abs(depth[cov] / z_ray - 1.0)
    assert rel.max() < 2e-4, rel.max()
    # a single constant-colour surface: the warped colour is that colour
    ref, _, _ = sc.shade(org[cov], d[cov], O.shading_params())
    assert np.abs(right[cov] - ref).max() < 1e-5


def _quads():
    def quad(z, half, k):
        vq = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], np.float32)
        return vq, np.array([[0, 1, 2], [0, 2, 3]], np.int32) + 4 * k
    vn, fn = quad(1.0, 0.3, 0)
    vf, ff = quad(3.0, 3.0, 1)
    return np.concatenate([vn, vf]), np.concatenate([fn, ff])


def test_depth_jumps_are_not_bridged_and_nearer_surfaces_win(O, layout):
    vv, ff = _quads()
    sc = O.Scene(vv, ff)
    cam = np.array([0, 0, -1, 1, 0, 0, 0, 1, 0, 0, 0, 1], np.float32)
    cr = cam.copy()
    cr[0] += 0.064
    W, H, gz = 640, 360, (320.0, 180.0)
    depth = np.zeros(layout.n_texels, np.float32)
    left, right, tri, fl, rid = O.rep_lp(sc, layout, W, H, I.FOV, gz, cam, cr, O.shading_params(), depth=depth)
    cov = (tri >= 0) & ~fl
    # the near quad is at depth 2, the far one at 4; nothing in between
    dz = depth[cov]
    assert np.all((np.abs(dz - 2.0) < 1e-3) | (np.abs(dz - 4.0) < 1e-3))
    G = O.gaze_film(W, H, O.film_pitch(W, H, *I.FOV), *gz)
    rid_ray = sc.closest(*O.vafr_rays(layout, np.arange(layout.n_texels), G, cr))[0]
    near = cov & (rid_ray >= 0) & (rid_ray <= 1)
    assert near.sum() > 1000
    # only along the quad's outline may the warp and the ray disagree
    assert np.mean(rid[near] <= 1) > 0.995
    # the disoccluded strip beside the near quad is left to ray casting
    assert ((tri < 0) & (rid_ray >= 2)).sum() > 100


def test_baseline_shifts_points_by_b_over_z(O, layout):
    """Right eye moved by b along +x: a point at depth z moves by -b / z on
    the right film, so a right texel's source texel sits b / z further +x."""
    vv = np.array([[-40, -40, 5], [40, -40, 5], [40, 40, 5], [-40, 40, 5]], np.float32)
    ff = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    sc = O.Scene(vv, ff)
    cam = np.array([0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1], np.float32)
    cr = cam.copy()
    b = 0.2
    cr[0] += b
    depth = np.zeros(layout.n_texels, np.float32)
    left, right, tri, fl, rid = O.rep_lp(sc, layout, 640, 360, I.FOV, (320.0, 180.0), cam, cr, O.shading_params(),
                                         depth=depth)
    cov = np.nonzero((tri >= 0) & ~fl)[0]
    x_src = layout.dxy[0::2][tri[cov] >> 1].astype(np.float64)
    x_dst = layout.dxy[0::2][cov].astype(np.float64)
    shift = np.mean(x_src - x_dst)
    assert abs(shift - b / 5.0) < 0.05 * b / 5.0, shift
    assert np.allclose(depth[cov], 5.0, rtol=1e-5)
