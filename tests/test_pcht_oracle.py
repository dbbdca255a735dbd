"""Pins of the PCHT oracle (pruned continuous Haar transform) against facts
fixed by the paper's definitions and by mathematics.

The paper prints no Haar coefficient values, so the pins are:

* brute force: every coefficient as the inner product of a rasterized tile
  with the basis function built from its definition (Sec. II-B: scaling
  function, Haar filters g and h, the wavelet as a filtered sum of
  finer scaling functions).  For lattice polygons the indicator is constant
  on unit pixels, so a pixel-centre raster gives the exact inner products
  (the paper notes that CHT and DHT coefficients coincide for such patterns);
* Parseval: the basis is orthonormal, so with unit cells at the finest level
  the squared coefficients sum to the area inside the tile;
* orientation and linearity (Sec. II-A2, Sec. III-A);
* the number of non-terminating calls for shapes where it is known.

A mistake in a filter sign, an x/y swap, a child order, the level factor
2^j / sqrt(Nx Ny) or the pyramid position breaks the brute-force pin.
"""
import numpy as np
import pytest

import synth


def _random_loops(rng, nx, ny, n_poly, spill=0):
    """Disjoint random polygons (unions of small rectangles) in a box that may
    stick out of [0,nx) x [0,ny) by ``spill``."""
    loops, taken = [], np.zeros((nx + 2 * spill, ny + 2 * spill), bool)
    tries = 0
    while len(loops) < n_poly and tries < 400:
        tries += 1
        n = int(rng.integers(1, 4))
        r = []
        for _ in range(n):
            x1 = int(rng.integers(-spill, nx + spill - 1))
            y1 = int(rng.integers(-spill, ny + spill - 1))
            x2 = int(rng.integers(x1 + 1, min(nx + spill, x1 + 1 + max(2, nx // 2)) + 1))
            y2 = int(rng.integers(y1 + 1, min(ny + spill, y1 + 1 + max(2, ny // 2)) + 1))
            r.append((x1, y1, x2, y2))
        lp = synth.loops_of_rect_union(r)
        if lp is None or len(lp) != 1:
            continue
        cov = np.zeros_like(taken)
        for (x1, y1, x2, y2) in r:
            cov[x1 + spill:x2 + spill, y1 + spill:y2 + spill] = True
        # keep polygons apart by one unit so that the union stays disjoint
        grown = cov.copy()
        grown[1:, :] |= cov[:-1, :]
        grown[:-1, :] |= cov[1:, :]
        grown[:, 1:] |= cov[:, :-1]
        grown[:, :-1] |= cov[:, 1:]
        if np.any(grown & taken):
            continue
        taken |= cov
        loops.append(lp[0])
    off = np.zeros(len(loops) + 1, np.int64)
    off[1:] = np.cumsum([p.shape[0] for p in loops])
    return np.concatenate(loops).astype(np.int64), off


def _raster(xy, off, nx, ny):
    """0/1 coverage of every unit pixel of the tile: even-odd test of the
    pixel centre against the vertical edges (a ray towards +x)."""
    img = np.zeros((nx, ny))
    cx = np.arange(nx) + 0.5
    cy = np.arange(ny) + 0.5
    X, Y = np.meshgrid(cx, cy, indexing="ij")
    for m in range(off.size - 1):
        p = xy[off[m]:off[m + 1]].astype(float)
        q = np.roll(p, -1, axis=0)
        inside = np.zeros_like(X, dtype=bool)
        for (xa, ya), (xb, yb) in zip(p, q):
            if xa != xb:
                continue
            lo, hi = min(ya, yb), max(ya, yb)
            inside ^= (xa > X) & (Y > lo) & (Y < hi)
        img += inside
    return img


def _phi(nx, ny, j, kx, ky):
    """phi_{j,kx,ky} sampled on unit pixels (Sec. II-B)."""
    b = np.zeros((nx, ny))
    wx, wy = nx >> j, ny >> j
    b[kx * wx:(kx + 1) * wx, ky * wy:(ky + 1) * wy] = 2.0 ** j / np.sqrt(nx * ny)
    return b


G_TAPS = np.array([1.0, 1.0]) / np.sqrt(2.0)
H_TAPS = np.array([1.0, -1.0]) / np.sqrt(2.0)


def _psi(nx, ny, j, kx, ky, a, b):
    """psi^{ab}_{j,kx,ky} = sum_n sum_m a_n b_m phi_{j+1, 2kx+n, 2ky+m}."""
    out = np.zeros((nx, ny))
    for n in range(2):
        for m in range(2):
            out += a[n] * b[m] * _phi(nx, ny, j + 1, 2 * kx + n, 2 * ky + m)
    return out


def _brute_pyramid(img, nx, ny, J):
    side = 1 << J
    W = np.zeros((side, side))
    W[0, 0] = np.sum(img * _phi(nx, ny, 0, 0, 0))
    for j in range(J):
        p = 1 << j
        for kx in range(p):
            for ky in range(p):
                W[ky, p + kx] = np.sum(img * _psi(nx, ny, j, kx, ky, H_TAPS, G_TAPS))
                W[p + ky, kx] = np.sum(img * _psi(nx, ny, j, kx, ky, G_TAPS, H_TAPS))
                W[p + ky, p + kx] = np.sum(img * _psi(nx, ny, j, kx, ky, H_TAPS, H_TAPS))
    return W


@pytest.mark.parametrize("nx,ny,J,seed,spill", [
    (16, 16, 4, 1, 0),
    (16, 16, 2, 2, 0),
    (32, 8, 3, 3, 0),
    (8, 16, 3, 4, 3),
    (16, 16, 4, 5, 4),
])
def test_pcht_matches_brute_force_inner_products(oracle_lib, nx, ny, J, seed, spill):
    rng = np.random.default_rng(seed)
    xy, off = _random_loops(rng, nx, ny, 4, spill)
    U, W, _ = oracle_lib.pcht(xy, off, nx, ny, J)
    Wb = _brute_pyramid(_raster(xy, off, nx, ny), nx, ny, J)
    assert np.max(np.abs(W - Wb)) <= 1e-12 * max(1.0, np.max(np.abs(Wb)))
    # U is W without the level factor, and an integer
    side = 1 << J
    lev = np.zeros((side, side), int)
    for r in range(side):
        for c in range(side):
            m = max(r, c)
            lev[r, c] = int(np.floor(np.log2(m))) if m else 0
    np.testing.assert_allclose(U * (2.0 ** lev) / np.sqrt(nx * ny), Wb, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_pcht_parseval(oracle_lib, seed):
    n, J = 64, 6
    rng = np.random.default_rng(seed)
    xy, off = _random_loops(rng, n, n, 6, spill=5)
    U, W, _ = oracle_lib.pcht(xy, off, n, n, J)
    area_in_tile = _raster(xy, off, n, n).sum()
    assert abs(np.sum(W * W) - area_in_tile) <= 1e-9 * area_in_tile
    assert U[0, 0] == area_in_tile


def test_pcht_orientation_and_linearity(oracle_lib):
    rng = np.random.default_rng(21)
    n, J = 128, 7
    xy, off = _random_loops(rng, n, n, 5, spill=6)
    U, _, nodes = oracle_lib.pcht(xy, off, n, n, J)
    # every loop reversed (counter-clockwise) describes the same set
    rev = np.concatenate([xy[off[m]:off[m + 1]][::-1] for m in range(off.size - 1)])
    U2, _, nodes2 = oracle_lib.pcht(rev, off, n, n, J)
    assert np.array_equal(U, U2) and nodes == nodes2
    # the transform of the set is the sum of the polygons' transforms
    acc = np.zeros_like(U)
    total = 0
    for m in range(off.size - 1):
        Um, _, nm = oracle_lib.pcht(xy[off[m]:off[m + 1]], np.array([0, off[m + 1] - off[m]]),
                                    n, n, J)
        acc += Um
        total += nm
    assert np.array_equal(U, acc) and nodes == total


def test_pcht_node_counts_of_simple_shapes(oracle_lib):
    # a rectangle equal to one level-1 cell: the root is the only cell that
    # meets the boundary without containing or missing the polygon
    sq = synth.rectangle_loop(0, 0, 32, 32).astype(np.int64)
    U, W, nodes = oracle_lib.pcht(sq, np.array([0, 4]), 64, 64, 6)
    assert nodes == 1
    assert U[0, 0] == 1024
    assert U[0, 1] == 1024 and U[1, 0] == 1024 and U[1, 1] == 1024  # hg, gh, hh of level 0
    assert np.count_nonzero(U) == 4
    # the whole tile: no wavelet sees a change
    full = synth.rectangle_loop(0, 0, 64, 64).astype(np.int64)
    U, _, nodes = oracle_lib.pcht(full, np.array([0, 4]), 64, 64, 6)
    assert nodes == 0 and U[0, 0] == 4096 and np.count_nonzero(U) == 1
    # a unit square at an odd position: one cell per level contains it
    px = synth.rectangle_loop(37, 21, 38, 22).astype(np.int64)
    U, W, nodes = oracle_lib.pcht(px, np.array([0, 4]), 64, 64, 6)
    assert nodes == 6
    assert abs(np.sum(W * W) - 1.0) <= 1e-12
    # outside the tile: nothing at all
    U, _, nodes = oracle_lib.pcht(px + 100, np.array([0, 4]), 64, 64, 6)
    assert nodes == 0 and not U.any()


def test_pcht_rejects_bad_input(oracle_lib):
    sq = synth.rectangle_loop(0, 0, 3, 3).astype(np.int64)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.pcht(sq, np.array([0, 4]), 24, 24, 4)  # 16 does not divide 24
    bad = np.array([[0, 0], [0, 2], [2, 3], [2, 0]])
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.pcht(bad, np.array([0, 4]), 16, 16, 2)
