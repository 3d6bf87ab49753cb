"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
its host layout tables equal the oracle's bit for bit, it validates
arguments, and its BVH is structurally sound.  No GPU compute here."""
import os
import re

import numpy as np
import pytest

from paper_2503_23410_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def V():
    from paper_2503_23410_amd import vafr
    vafr.load()
    return vafr


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "vafr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", src, flags=re.M)
    return {n for n in names if n not in ("if", "defined")}


def test_library_exports_every_declared_symbol(V):
    declared = _declared_functions()
    assert declared == set(V.EXPORTS)
    lib = V.load()
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.vafr_abi_version() == 2


def test_vafr_layout_tables_bit_exact_with_oracle(V, O, layout):
    for W, H in ((640, 360), (7680, 4320)):
        L = V.Layout.vafr(V.display(W, H))
        assert (L.n_cols, L.n_texels) == (layout.n_cols, layout.n_texels)
        n_rows, col_off, dxy = L.tables()
        assert np.array_equal(n_rows, layout.n_rows)
        assert np.array_equal(col_off, layout.col_off)
        assert np.array_equal(dxy.view(np.uint32), layout.dxy.view(np.uint32))
        assert L.max_rows == layout.n_rows.max()


def test_custom_acuity_layout_matches_oracle(V, O):
    """Device-adapted pivots (Sec. 3.3: other curves are just other pivot
    values) go through the same code; tables still match bit for bit."""
    ecc, cpd = (0.0, 10.0, 20.0, 30.0, 60.0), (9.0, 9.0, 6.0, 5.0, 4.0)
    L = V.Layout.vafr(V.display(1920, 1080), ecc, cpd, 60.0)
    ref = O.Layout(O.Acuity(ecc, cpd), 60.0)
    n_rows, col_off, dxy = L.tables()
    assert np.array_equal(n_rows, ref.n_rows) and np.array_equal(col_off, ref.col_off)
    assert np.array_equal(dxy.view(np.uint32), ref.dxy.view(np.uint32))
    assert L.n_texels < 1061735 * 0.85   # capping f at 9 cpd removes work


@pytest.mark.parametrize("cap,aniso", [(9.0, None), (18.0, None), (None, ([0.0, 30.0], [1.0, 0.5])),
                                       (9.0, ([0.0, 15.0, 45.0], [1.0, 0.6, 0.4])), (None, ([0.0, 60.0], [1.0, 1.0]))])
def test_device_curve_and_anisotropic_layouts_match_oracle(V, O, cap, aniso):
    """Device-adapted pivots (min(f, cap), Sec. 3.3) and the anisotropic row
    counts of Eq. (19): the library's pivots and tables equal the oracle's
    bit for bit."""
    if cap is None:
        ecc, cpd = O.DEFAULT_ECC, (40.0, 10.0, 6.0, 5.0, 4.0)
    else:
        ecc, cpd = V.acuity_capped(cap)
        eo, co = O.acuity_capped(cap)
        assert np.array_equal(ecc, eo) and np.array_equal(cpd, co)
    L = V.Layout.vafr(V.display(1920, 1080), ecc, cpd, 60.0, aniso=aniso)
    ref = O.Layout(O.Acuity(ecc, cpd, aniso=aniso), 60.0)
    n_rows, col_off, dxy = L.tables()
    assert (L.n_cols, L.n_texels) == (ref.n_cols, ref.n_texels)
    assert np.array_equal(n_rows, ref.n_rows) and np.array_equal(col_off, ref.col_off)
    assert np.array_equal(dxy.view(np.uint32), ref.dxy.view(np.uint32))


@pytest.mark.parametrize("aniso", [([0.0, 0.0], [1.0, 1.0]), ([0.0, 30.0], [1.0, 0.0]), ([0.0], [17.0]),
                                   ([0.0, float("nan")], [1.0, 1.0])])
def test_anisotropy_validation(V, aniso):
    with pytest.raises(V.VafrError) as ei:
        V.Layout.vafr(V.display(640, 360), aniso=aniso)
    assert ei.value.code == V.VAFR_E_ARG


def test_capped_curve_validation(V):
    for cap in (0.0, -1.0, float("inf")):
        with pytest.raises(V.VafrError):
            V.acuity_capped(cap)
    with pytest.raises(V.VafrError):
        V.acuity_capped(9.0, (1.0, 10.0), (40.0, 10.0))          # first pivot not at 0


def test_lmfr_layout_dims_match_oracle(V, O):
    for W, H in ((640, 360), (1920, 1080), (7680, 4320), (11520, 6480)):
        L = V.Layout.lmfr(V.display(W, H), 1.8, 4.0)
        assert (L.n_cols, L.max_rows) == O.lmfr_dims(W, H, 1.8)
        assert L.kind == V.VAFR_LAYOUT_LMFR
        n_rows, col_off, dxy = L.tables()
        assert dxy is None and np.all(n_rows == L.max_rows)


@pytest.mark.parametrize("bad", [
    dict(disp=(0, 100)), dict(disp=(100, -1)), dict(fov=(0.0, 90.0)), dict(fov=(90.0, 180.0)),
    dict(ecc=(1.0, 10.0), cpd=(40.0, 10.0)), dict(ecc=(0.0, 10.0, 10.0), cpd=(40.0, 10.0, 5.0)),
    dict(ecc=(0.0, 10.0), cpd=(40.0, 0.0)), dict(e_max=95.0), dict(ecc=(0.0, 10.0), cpd=(1.0, 2.0)),
])
def test_layout_argument_validation(V, bad):
    disp = V.display(*(bad.get("disp", (640, 360))), fov=bad.get("fov", (100.0, 100.0)))
    with pytest.raises(V.VafrError) as ei:
        V.Layout.vafr(disp, bad.get("ecc", (0.0, 10.0, 20.0, 30.0, 60.0)), bad.get("cpd", (40.0, 10.0, 6.0, 5.0, 4.0)),
                      bad.get("e_max", 60.0))
    assert ei.value.code == V.VAFR_E_ARG
    assert V.last_error()


def test_lmfr_argument_validation(V):
    for delta, alpha in ((0.5, 4.0), (1.8, 0.0), (float("nan"), 4.0)):
        with pytest.raises(V.VafrError) as ei:
            V.Layout.lmfr(V.display(640, 360), delta, alpha)
        assert ei.value.code == V.VAFR_E_ARG


def test_lafr_layout_dims_match_oracle(V, O):
    """LaFR(delta) shades the same (W/delta) x (H/delta) buffer as LMFR."""
    for W, H in ((640, 360), (1920, 1080), (7680, 4320), (11520, 6480)):
        for delta in (1.8, 2.2):
            L = V.Layout.lafr(V.display(W, H), delta)
            assert (L.n_cols, L.max_rows) == O.lmfr_dims(W, H, delta)
            assert L.kind == V.VAFR_LAYOUT_LAFR
            n_rows, col_off, dxy = L.tables()
            assert dxy is None and np.all(n_rows == L.max_rows)


def test_lafr_argument_validation(V):
    for delta, a, alpha, beta in ((0.5, 0.25, 0.85, 0.7), (1.8, 0.0, 0.85, 0.7), (1.8, 1.0, 0.85, 0.7),
                                  (1.8, 0.25, 0.0, 0.7), (1.8, 0.25, 1.5, 0.7), (1.8, 0.25, 0.85, 0.0),
                                  (float("nan"), 0.25, 0.85, 0.7)):
        with pytest.raises(V.VafrError) as ei:
            V.Layout.lafr(V.display(640, 360), delta, a, alpha, beta)
        assert ei.value.code == V.VAFR_E_ARG


def test_lafr_parameters_match_the_oracle(V, O):
    """The binding's default LaFR parameters are the oracle's."""
    assert (V.LAFR_A, V.LAFR_ALPHA, V.LAFR_BETA) == (O.LAFR_A, O.LAFR_ALPHA, O.LAFR_BETA)


def _check_bvh(V, verts, tris):
    sc = V.Scene(verts, tris)
    info = sc.info()
    nodes, order = sc.export()
    assert info["n_tris"] == tris.shape[0]
    assert np.array_equal(np.sort(order), np.arange(tris.shape[0]))      # each triangle stored once
    # binary build depth within the LDS class; the 4-wide collapse within
    # the LDS class plus the 24 spill entries
    assert info["stack_entries"] in (24, 32) and info["max_depth"] <= info["stack_entries"] - 1
    assert info["max_stack"] <= info["stack_entries"] + 24
    refs = nodes[:, 12:16].view(np.int32) if nodes.size else np.zeros((0, 4), np.int32)
    kids = (refs != np.iinfo(np.int32).min).sum(axis=1) if nodes.size else np.zeros(0, np.int64)
    tv = verts[tris[order]]                                               # stored order, (n, 3, 3)
    empty = np.iinfo(np.int32).min
    seen = np.zeros(len(nodes), int)

    def tri_range(ref):
        if ref < 0:
            x = ~ref
            return [(x >> 3, (x & 7) + 1)]
        seen[ref] += 1
        out = []
        for c in refs[ref]:
            if c != empty:
                out += tri_range(c)
        return out

    def planes(ni):
        """Decoded child planes (4 children x (lo, hi) x 3 axes) as the
        traversal's fallback computes them: fmaf(code, scale, origin)."""
        codes = nodes[ni, 4:12].view(np.uint32)
        scales = (float(nodes[ni, 10]), float(nodes[ni, 11]), float(nodes[ni, 3]))
        out = np.zeros((4, 2, 3))
        for a in range(3):
            scale = scales[a]
            assert scale > 0 and np.frexp(scale)[0] == 0.5          # a power of two
            for c in range(4):
                for side in range(2):
                    q = (int(codes[2 * a + side]) >> (8 * c)) & 255
                    out[c, side, a] = np.float32(np.float64(q) * scale + np.float64(nodes[ni, a]))
        return out

    # every triangle is reached exactly once from the root
    if info["n_nodes"]:
        ranges = tri_range(0)
        covered = np.zeros(tris.shape[0], int)
        for first, cnt in ranges:
            covered[first:first + cnt] += 1
        assert np.all(covered == 1) and np.all(seen == 1)
    # stack bound: the sum of (children - 1) along any root-to-node path
    worst = 0
    todo = [(0, 0)] if info["n_nodes"] else []
    while todo:
        n, used = todo.pop()
        below = used + kids[n] - 1
        worst = max(worst, below)
        todo += [(c, below) for c in refs[n] if c >= 0]
    assert worst == info["max_stack"]
    for ni in range(min(len(nodes), 2000)):
        k = kids[ni]
        assert 2 <= k <= 4
        assert np.all(refs[ni, k:] == empty) and np.all(refs[ni, :k] != empty)
        pl = planes(ni)
        for ch in range(k):
            lo, hi = pl[ch, 0], pl[ch, 1]
            for first, cnt in tri_range(refs[ni, ch]):
                pts = tv[first:first + cnt].reshape(-1, 3)
                assert np.all(pts >= lo) and np.all(pts <= hi)
    return sc, info


def test_bvh_structure_soup(V):
    v, f = I.soup_scene()
    sc, info = _check_bvh(V, v, f)
    assert info["n_leaves"] >= 4096 // 4


def test_bvh_structure_terrain_and_degenerate(V):
    v, f = I.terrain_scene(48, 24, 8, seed=4)
    _check_bvh(V, v, f)
    # many identical triangles force the depth guard and median splits
    tri = np.array([[0, 0, 1], [1, 0, 1], [0, 1, 1]], np.float32)
    vv = np.tile(tri, (3000, 1))
    ff = np.arange(9000, dtype=np.int32).reshape(-1, 3)
    sc, info = _check_bvh(V, vv, ff)
    assert info["stack_entries"] == 24 and info["max_depth"] <= 23


def test_bvh_small_and_empty_scenes(V):
    v, f = I.soup_scene(1, seed=1)
    sc = V.Scene(v, f)
    assert sc.info()["n_nodes"] == 0        # a single leaf at the root
    v, f = I.soup_scene(3, seed=1)
    _check_bvh(V, v, f)
    sc0 = V.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32))
    assert sc0.info()["n_tris"] == 0


def test_scene_validation(V):
    v, f = I.soup_scene(4, seed=1)
    bad = f.copy()
    bad[1, 2] = 99
    with pytest.raises(V.VafrError) as ei:
        V.Scene(v, bad)
    assert ei.value.code == V.VAFR_E_ARG
    vn = v.copy()
    vn[2, 1] = np.nan
    with pytest.raises(V.VafrError):
        V.Scene(vn, f)


def test_large_scene_bvh_builds_fast(V):
    v, f = I.make_scene("terrain1m")
    sc = V.Scene(v, f)
    info = sc.info()
    assert info["stack_entries"] == 24 and info["max_depth"] <= 23
    assert info["build_ms"] < 30000


@pytest.mark.slow
def test_stack_class_follows_scene_size(V):
    """Scenes of more than 2^23 triangles get the long stack class; the
    depth bound holds for both classes, also under forced median splits."""
    n = (1 << 23) + 4096
    rng = np.random.default_rng(9)
    c = rng.random((n, 3), dtype=np.float32) * 100.0
    vv = np.repeat(c, 3, axis=0)
    vv[1::3, 0] += 0.01
    vv[2::3, 1] += 0.01
    ff = np.arange(3 * n, dtype=np.int32).reshape(-1, 3)
    sc = V.Scene(vv, ff)
    info = sc.info()
    assert info["stack_entries"] == 32 and info["max_depth"] <= 31
    del sc, vv, ff
    # identical triangles: no SAH split applies, every level is a median split
    vv = np.tile(np.array([[0, 0, 1], [1, 0, 1], [0, 1, 1]], np.float32), ((1 << 21) + 17, 1))
    ff = np.arange(vv.shape[0], dtype=np.int32).reshape(-1, 3)
    info = V.Scene(vv, ff).info()
    assert info["stack_entries"] == 24 and info["max_depth"] <= 23
