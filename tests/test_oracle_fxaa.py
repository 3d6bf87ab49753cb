"""Pins for the oracle's FXAA-style anti-aliasing inside the LP buffer
(Sec. 3.4).  The paper names the method only; the checks fix what any
reading of it must do: flat and gently varying buffers pass unchanged,
every output is a blend of a texel with one of its neighbours, hard edges
are softened only next to the edge, an isolated bright texel is damped."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def grid(O):
    L = O.Layout()
    col = np.repeat(np.arange(L.n_cols), L.n_rows)                 # column of every texel
    row = np.arange(L.n_texels) - L.col_off[col]
    turns = (row + 0.5) / L.n_rows[col]
    return L, col, row, turns


def _lp(values):
    out = np.zeros((values.size, 4), np.float32)
    out[:, 0] = out[:, 1] = out[:, 2] = values
    out[:, 3] = 1.0
    return out


def test_flat_buffer_is_unchanged(O, grid):
    L, col, row, turns = grid
    lp = np.tile(np.float32([0.3, 0.5, 0.2, 1.0]), (L.n_texels, 1))
    assert np.array_equal(O.fxaa_lp(L, lp), lp)


def test_gentle_gradient_is_below_the_contrast_threshold(O, grid):
    """A ramp along the radius of 1/200 per column never reaches the
    contrast threshold (1/16 or 1/8 of the local maximum)."""
    L, col, row, turns = grid
    lp = _lp((col / 200.0).astype(np.float32) % 1.0)
    lp[col >= 200, :3] = 0.99                                         # keep the ramp monotone
    out = O.fxaa_lp(L, lp)
    keep = (col < 195) | (col > 205)
    assert np.array_equal(out[keep], lp[keep])


def _neighbour_values(L, lp, col, row, turns):
    """The four direct neighbours of every texel: rows j-1, j+1 of its own
    column, and the inner / outer columns at its angle (linear in rows)."""
    def at(c, t):
        c = np.clip(c, 0, L.n_cols - 1)
        n = L.n_rows[c]
        s = t * n - 0.5
        j0 = np.floor(s).astype(np.int64)
        w = (s - j0)[:, None]
        a = lp[L.col_off[c] + np.mod(j0, n)]
        b = lp[L.col_off[c] + np.mod(j0 + 1, n)]
        return a + w * (b - a)
    n = L.n_rows[col]
    return [lp[L.col_off[col] + np.mod(row - 1, n)], lp[L.col_off[col] + np.mod(row + 1, n)],
            at(col - 1, turns), at(col + 1, turns)]


def test_output_blends_a_texel_with_one_neighbour(O, grid):
    """Every output is centre + a (neighbour - centre) with one 0 <= a <= 1
    common to the four channels, for one of the four direct neighbours."""
    L, col, row, turns = grid
    rng = np.random.default_rng(7)
    lp = np.repeat(rng.random(L.n_texels, dtype=np.float32)[:, None], 4, axis=1) * np.float32([1.0, 0.8, 0.6, 1.0])
    lp = lp.astype(np.float32)
    out = O.fxaa_lp(L, lp)
    ok = np.all(np.abs(out - lp) <= 1e-7, axis=1)
    for nb in _neighbour_values(L, lp, col, row, turns):
        d = nb - lp
        a = np.where(np.abs(d[:, 0]) > 1e-6, (out[:, 0] - lp[:, 0]) / np.where(d[:, 0] == 0, 1, d[:, 0]), 0.0)
        fit = np.all(np.abs(lp + a[:, None] * d - out) <= 2e-6, axis=1) & (a >= -1e-6) & (a <= 1 + 1e-6)
        ok |= fit
    assert ok.mean() > 0.999, ok.mean()


def test_edge_across_the_radius_softens_only_next_to_it(O, grid):
    """Columns below 300 dark, from 300 on bright: the edge runs along the
    angle.  Only columns 299 and 300 change, toward the other side, within
    [0, 1]; the bright side of the step stays above the dark side."""
    L, col, row, turns = grid
    lp = _lp(np.where(col < 300, 0.0, 1.0).astype(np.float32))
    out = O.fxaa_lp(L, lp)
    changed = np.any(out != lp, axis=1)
    assert set(np.unique(col[changed])) <= {299, 300}
    assert changed[col == 299].mean() > 0.9 and changed[col == 300].mean() > 0.9
    assert np.all(out[col == 299, 0] > 0.0) and np.all(out[col == 300, 0] < 1.0)
    assert out[col == 299, 0].max() < out[col == 300, 0].min()
    assert np.all((out >= 0.0) & (out <= 1.0))


def test_edge_across_the_angle_softens_only_next_to_it(O, grid):
    """Half of every column (angles in [0, 1/2)) dark, the other half bright:
    the edge runs along the radius.  Only texels at most one row from the
    two seam angles change; far texels keep their value."""
    L, col, row, turns = grid
    lp = _lp(np.where(turns < 0.5, 0.0, 1.0).astype(np.float32))
    out = O.fxaa_lp(L, lp)
    changed = np.any(out != lp, axis=1)
    n = L.n_rows[col]
    rows_from_seam = np.minimum(np.abs(turns - 0.5), np.minimum(turns, 1.0 - turns)) * n
    big = n >= 16
    assert np.all(~changed[big & (rows_from_seam > 1.01)])
    assert changed[big & (rows_from_seam < 0.51)].mean() > 0.9
    assert np.all((out >= 0.0) & (out <= 1.0))


def test_isolated_bright_texel_is_damped(O, grid):
    """Sub-texel aliasing: one bright texel in a dark field loses luma to its
    neighbourhood; its neighbours are not brightened beyond it."""
    L, col, row, turns = grid
    vals = np.zeros(L.n_texels, np.float32)
    k = L.col_off[400] + 500
    vals[k] = 1.0
    lp = _lp(vals)
    out = O.fxaa_lp(L, lp)
    assert 0.0 < out[k, 0] < 0.6
    assert np.all(out[:, 0] <= out[k, 0] + 1e-6)
