"""The allocation-free reprojection entry point (vafr_shade_lp_rep_noalloc,
workspace in the library's static device array) gives exactly the results
of vafr_shade_lp_rep with a caller workspace: two calls in a row, the second
on a smaller layout, with the static array holding the first call's
contents.  Oversized layouts and layouts whose tables are not yet on the
device are refused before any launch."""
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


def _bufs(torch, n, fill):
    lp = torch.full((n, 4), fill, device="cuda")
    hid = torch.full((n,), -5, device="cuda", dtype=torch.int32)
    return lp, hid


def test_noalloc_rep_equals_workspace_rep(env):
    torch, V = env
    v, f = I.make_scene("terrain1m")
    sc = V.Scene(v, f)
    W, H = 1920, 1080
    cl, cr = I.binocular_cameras()
    sh = V.shading()
    ecc9, cpd9 = V.acuity_capped(9.0)
    layouts = [V.Layout.vafr(V.display(W, H)), V.Layout.vafr(V.display(W, H), ecc9, cpd9, 60.0)]
    assert layouts[1].n_texels < layouts[0].n_texels
    for call, (L, gz) in enumerate(zip(layouts, ((900.0, 500.0), (1200.0, 300.0)))):
        n = L.n_texels
        log(f"call {call}: {n} texels, gaze {gz}")
        ll, hl = _bufs(torch, n, -1.0)
        lr, hr = _bufs(torch, n, -1.0)
        ws = torch.empty(V.rep_workspace_bytes(L), device="cuda", dtype=torch.uint8)
        V.vafr_shade_lp_rep(sc, V.camera(cl), V.camera(cr), V.gaze(*gz), sh, L, ll, lr, ws, hl, hr)
        torch.cuda.synchronize()
        nl, nhl = _bufs(torch, n, -3.0)
        nr, nhr = _bufs(torch, n, -3.0)
        V.vafr_shade_lp_rep_noalloc(sc, V.camera(cl), V.camera(cr), V.gaze(*gz), sh, L, nl, nr, nhl, nhr)
        torch.cuda.synchronize()
        assert torch.equal(nl, ll) and torch.equal(nhl, hl), f"call {call}: left eye differs"
        assert torch.equal(nr, lr) and torch.equal(nhr, hr), f"call {call}: right eye differs"
        assert int((hr >= 0).sum()) > n // 2
        log(f"call {call}: left and right LP buffers and hit ids equal the workspace call")


def test_noalloc_rep_refusals(env):
    torch, V = env
    v, f = I.soup_scene()
    sc = V.Scene(v, f)
    cl = I.soup_camera()
    cr = cl.copy()
    cr[0] += 0.064
    sh = V.shading()
    # twice the paper's acuity: about four times the texels, beyond the static workspace
    big = V.Layout.vafr(V.display(640, 360), (0.0, 10.0, 20.0, 30.0, 60.0), (80.0, 20.0, 12.0, 10.0, 8.0), 60.0)
    lp = torch.empty((big.n_texels, 4), device="cuda")
    with pytest.raises(V.VafrError) as e:
        V.vafr_shade_lp_rep_noalloc(sc, V.camera(cl), V.camera(cr), V.gaze(320.0, 180.0), sh, big, lp, lp.clone())
    assert e.value.code == V.VAFR_E_BUDGET
    # a fresh layout has no tables on the device yet: refused, then accepted
    # once a per-frame call has uploaded them
    L = V.Layout.vafr(V.display(640, 360))
    a, b = torch.empty((L.n_texels, 4), device="cuda"), torch.empty((L.n_texels, 4), device="cuda")
    with pytest.raises(V.VafrError) as e:
        V.vafr_shade_lp_rep_noalloc(sc, V.camera(cl), V.camera(cr), V.gaze(320.0, 180.0), sh, L, a, b)
    assert e.value.code == V.VAFR_E_UNSUPPORTED
    V.vafr_shade_lp(sc, V.camera(cl), V.gaze(320.0, 180.0), sh, L, a)
    V.vafr_shade_lp_rep_noalloc(sc, V.camera(cl), V.camera(cr), V.gaze(320.0, 180.0), sh, L, a, b)
    torch.cuda.synchronize()
