"""Pins of the oracle's mask-given grain (marching-squares boundary over the
cell centres at level 1/2, even-odd inside): the cells it encloses are the
mask's, saddle squares keep their diagonal corners apart, a block of cells
has trajectory segments in closed form, and a mask sampled from a disc has
chords within two cells (one per end) of the disc's."""
import math

import numpy as np
import pytest

from oracle import geometry as geo


@pytest.mark.parametrize("seed", range(6))
def test_mask_encloses_exactly_its_cells(seed):
    rng = np.random.default_rng(seed)
    nx, ny = int(rng.integers(5, 17)), int(rng.integers(5, 17))
    g = geo.Grid(nx, ny, float(rng.uniform(0.3, 0.9)), x0=float(rng.uniform(-3, 1)), y0=float(rng.uniform(-3, 1)))
    m = rng.random((ny, nx)) < rng.uniform(0.3, 0.7)
    sh = geo.MaskShape(m, g)
    X, Y = g.centres()
    assert np.array_equal(sh.inside(X, Y), m)


def test_checkerboard_and_saddles():
    g = geo.Grid(6, 5, 1.0, 0.0, 0.0)
    m = (np.add.outer(np.arange(5), np.arange(6)) % 2) == 0
    sh = geo.MaskShape(m, g)
    X, Y = g.centres()
    assert np.array_equal(sh.inside(X, Y), m)
    # the centre of a square between four centres is outside: the two
    # diagonal inside corners are not joined
    xs = g.x0 + np.arange(1, 6) * g.h
    ys = g.y0 + np.arange(1, 5) * g.h
    XX, YY = np.meshgrid(xs, ys)
    assert not sh.inside(XX, YY).any()
    # each inside cell is cut off by four diagonal pieces (a diamond)
    assert len(sh.ax) == 4 * int(m.sum())


@pytest.mark.parametrize("phi", [0.0, 0.5 * math.pi])
def test_block_of_cells_segments_closed_form(phi):
    nx, ny, h = 12, 10, 0.5
    g = geo.Grid(nx, ny, h)
    i0, i1, j0, j1 = 3, 8, 2, 6
    m = np.zeros((ny, nx), dtype=bool)
    m[j0:j1 + 1, i0:i1 + 1] = True
    sh = geo.MaskShape(m, g)
    tb = geo.AngleTable(g, [sh], phi)
    half = 0.5 * (tb.M - 1)
    got = {}
    for s in range(tb.nseg):
        got[int(tb.seg_line[s])] = (tb.smin[s], tb.smax[s])
    # the lines through the block's centre rows (phi = 0) or columns
    # (phi = pi/2) run from one vertical (horizontal) side of the contour,
    # half a cell outside the outer centres, to the other
    if phi == 0.0:
        lo, hi = g.x0 + i0 * h - g.cx, g.x0 + (i1 + 1) * h - g.cx
        rows = [(g.cy - (g.y0 + (j + 0.5) * h)) / h + half for j in range(j0, j1 + 1)]
    else:
        lo, hi = g.y0 + j0 * h - g.cy, g.y0 + (j1 + 1) * h - g.cy
        rows = [((g.x0 + (i + 0.5) * h) - g.cx) / h + half for i in range(i0, i1 + 1)]
    for r in rows:
        line = int(round(r))
        assert abs(r - line) < 1e-9
        s0, s1 = got[line]
        assert abs(s0 - lo) < 1e-12 and abs(s1 - hi) < 1e-12


def test_mask_of_a_disc_has_chords_within_two_cells():
    nx, ny, h, R = 48, 48, 0.25, 4.3
    g = geo.Grid(nx, ny, h)
    X, Y = g.centres()
    m = X * X + Y * Y <= R * R
    disc = geo.Disc(0.0, 0.0, R)
    sh = geo.MaskShape(m, g)
    for phi in (0.0, 0.3, 1.1):
        tm = geo.AngleTable(g, [sh], phi)
        td = geo.AngleTable(g, [disc], phi)
        ld = {int(td.seg_line[s]): td.smax[s] - td.smin[s] for s in range(td.nseg)}
        lm = {}
        for s in range(tm.nseg):
            lm[int(tm.seg_line[s])] = lm.get(int(tm.seg_line[s]), 0.0) + tm.smax[s] - tm.smin[s]
        common = set(ld) & set(lm)
        assert len(common) >= 0.9 * len(ld)
        assert max(abs(ld[k] - lm[k]) for k in common) <= 2.0 * h
