"""Properties of the seeded layout generator (no Fourier arithmetic here)."""
import numpy as np
import pytest

import synth
from tests import helpers as H


def _check_loops(xy, off, vmin=4, vmax=40):
    xy = np.asarray(xy, dtype=np.int64)
    for m in range(len(off) - 1):
        p = xy[off[m]:off[m + 1]]
        n = p.shape[0]
        assert vmin <= n <= vmax and n % 2 == 0
        q = np.roll(p, -1, axis=0)
        horiz = p[:, 1] == q[:, 1]
        vert = p[:, 0] == q[:, 0]
        assert np.all(horiz ^ vert)                       # axis-parallel, nonzero
        assert np.all(horiz != np.roll(horiz, -1))        # alternating
        assert H.shoelace2(p, [0, n])[0] < 0              # clockwise (y up)


def test_clip_recipe_and_determinism():
    c = synth.clip(2, 4096, 255, n_polygons=300)
    assert c.n_loops == 300
    _check_loops(c.xy, c.off)
    assert c.xy.min() >= 0 and c.xy.max() <= 4096
    c2 = synth.clip(2, 4096, 255, n_polygons=300)
    assert np.array_equal(c.xy, c2.xy) and np.array_equal(c.off, c2.off)
    c3 = synth.clip(3, 4096, 255, n_polygons=300)
    assert not np.array_equal(c.xy[:100], c3.xy[:100])


def test_clip_min_vertices():
    c = synth.clip(9, 8192, 511, min_vertices=5000)
    assert 5000 <= c.n_vertices < 5040
    _check_loops(c.xy, c.off)


def test_disjoint_clip_has_no_overlap():
    c = synth.clip(4, 1024, 63, n_polygons=60, disjoint=True)
    _check_loops(c.xy, c.off)
    img = H.raster(c.xy, c.off, 1024)
    assert img.max() == 1  # no two polygons share a cell


def test_c1_single_polygon():
    c, sub, nr = synth.clip_c1(1)
    assert c.n_loops == 1 and c.n_vertices == 64 and nr >= 8
    _check_loops(c.xy, c.off, 64, 64)
    assert c.xy.min() >= 0 and c.xy.max() < 2048


def test_union_loops_match_raster():
    rects = [(2, 3, 20, 9), (10, 5, 15, 30), (12, 25, 40, 33)]
    loops = synth.loops_of_rect_union(rects)
    assert len(loops) == 1
    img = np.zeros((64, 64), np.int64)
    for x1, y1, x2, y2 in rects:
        img[x1:x2, y1:y2] = 1
    assert np.array_equal(H.raster(loops[0], [0, loops[0].shape[0]], 64), img)
    # a saddle (two cells touching at a corner) is rejected
    assert synth.loops_of_rect_union([(0, 0, 5, 5), (5, 5, 9, 9)]) is None


def test_batch_clips():
    cl = synth.batch_clips(4, n_clips=6, v_lo=1000, v_hi=5000, pool=64)
    assert len(cl) == 6
    for c in cl:
        assert (c.T, c.K) in synth.layouts.BATCH_TK
        assert 1000 <= c.n_vertices <= 5000 + 40
        _check_loops(c.xy, c.off)
        assert c.xy.min() >= 0 and c.xy.max() <= c.T
