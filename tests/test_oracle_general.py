"""Pins of the general-tile oracle (periods Nx != Ny, any integers, vertices on
the grid of step 2^-F) against facts fixed by the paper's definitions and by
mathematics, independent of the oracle's own formula:

* a rectangle with fractional corners on a non-square, non-power-of-two tile
  against direct integration of the Fourier basis of Sec. II-C (a product of
  two 1-D integrals);
* a union of half-unit cells (fractional lattice) against the sum of the
  cells' closed forms, by brute force;
* scaling: the same polygons drawn at half size with F = 1 on a tile of half
  the periods have exactly half the coefficients (substitution in the
  integral), which pins both the fractional phases and the sqrt factors of
  alpha;
* a square power-of-two tile with F = 0 agrees with the square-tile oracle.

A slip in any of the four alpha factors (sqrt(Nx/Ny) and sqrt(Ny/Nx) swapped,
1/sqrt(Nx Ny) for the DC term), in the period used for each axis, or in the
fractional phase reduction breaks one of them.
"""
import numpy as np
import pytest

import synth
from tests import helpers as H


def _rect_general(x1, y1, x2, y2, Nx, Ny, K, L):
    k = np.arange(-K, K + 1)
    l = np.arange(-L, L + 1)
    Ix = H.rect_interval(x1, x2, k, Nx)
    Iy = H.rect_interval(y1, y2, l, Ny)
    return np.outer(Ix, Iy) / np.sqrt(Nx * Ny)


def _loop(x1, y1, x2, y2):
    return np.array([[x1, y1], [x1, y2], [x2, y2], [x2, y1]], dtype=np.float64), np.array([0, 4])


@pytest.mark.parametrize("Nx,Ny,F", [(50, 36, 0), (50, 36, 2), (37, 64, 3), (4096, 1000, 1)])
def test_general_rectangle_against_direct_integration(oracle_lib, Nx, Ny, F):
    # corners on the grid of step 2^-F
    x1, y1, x2, y2 = (np.floor(v * 2 ** F) / 2 ** F for v in (3.375, 5.625, 20.875, 31.0))
    xy, off = _loop(x1, y1, x2, y2)
    K, L = 9, 6
    Fo, area = oracle_lib.cfs_grid_general(xy, off, Nx, Ny, K, L, frac_bits=F)
    G = _rect_general(x1, y1, x2, y2, Nx, Ny, K, L)
    assert np.max(np.abs(Fo - G)) <= 1e-13 * abs(G[K, L])
    assert area == round((x2 - x1) * (y2 - y1) * 4 ** F)
    assert abs(Fo[K, L] - (x2 - x1) * (y2 - y1) / np.sqrt(Nx * Ny)) <= 1e-15 * Nx * Ny


def test_general_half_cell_union_brute_force(oracle_lib):
    # random union of half-unit cells on a 9 x 7 tile (fractional grid, F = 1)
    rng = np.random.default_rng(5)
    Nx, Ny, F = 9, 7, 1
    rects = []
    for _ in range(5):
        x1, y1 = rng.integers(0, 2 * Nx - 4), rng.integers(0, 2 * Ny - 4)
        rects.append((x1, y1, x1 + rng.integers(1, 5), y1 + rng.integers(1, 5)))
    loops = synth.loops_of_rect_union(rects)
    assert loops is not None
    off = np.zeros(len(loops) + 1, np.int64)
    off[1:] = np.cumsum([p.shape[0] for p in loops])
    xy_half = np.concatenate(loops).astype(np.float64) / 2.0
    K, L = 6, 5
    Fo, _ = oracle_lib.cfs_grid_general(xy_half, off, Nx, Ny, K, L, frac_bits=F)
    # brute force: every covered half-cell integrates to a product of 1-D integrals
    occ = np.zeros((2 * Nx, 2 * Ny), bool)
    for (a, b, c, d) in rects:
        occ[a:c, b:d] = True
    k = np.arange(-K, K + 1)
    l = np.arange(-L, L + 1)
    G = np.zeros((2 * K + 1, 2 * L + 1), complex)
    for i, j in zip(*np.nonzero(occ)):
        G += np.outer(H.rect_interval(i / 2, (i + 1) / 2, k, Nx),
                      H.rect_interval(j / 2, (j + 1) / 2, l, Ny))
    G /= np.sqrt(Nx * Ny)
    assert np.max(np.abs(Fo - G)) <= 1e-12 * abs(G[K, L])


@pytest.mark.parametrize("Nx,Ny", [(300, 200), (256, 512)])
def test_general_half_scale_halves_the_coefficients(oracle_lib, Nx, Ny):
    clip = synth.clip(12, min(Nx, Ny), 8, n_polygons=6)
    K, L = 8, 7
    F1, a1 = oracle_lib.cfs_grid_general(clip.xy.astype(float), clip.off, Nx, Ny, K, L)
    F2, a2 = oracle_lib.cfs_grid_general(clip.xy.astype(float) / 2, clip.off, Nx // 2, Ny // 2,
                                         K, L, frac_bits=1)
    assert np.max(np.abs(F2 - F1 / 2)) <= 1e-12 * abs(F1[K, L])
    assert a1 == a2  # area times 4^F: the same integer


def test_general_square_tile_matches_square_oracle(oracle_lib):
    clip = synth.clip(13, 128, 10, n_polygons=20)
    Fg, ag = oracle_lib.cfs_grid_general(clip.xy.astype(float), clip.off, 128, 128, 10, 9)
    Fs, as_ = oracle_lib.cfs_grid(clip.xy, clip.off, 128, 10, 9)
    assert np.max(np.abs(Fg - Fs)) <= 1e-13 * abs(Fs[10, 9]) and ag == as_


def test_general_rejects_off_grid_coordinates(oracle_lib):
    xy, off = _loop(0.25, 0, 3, 2)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.cfs_grid_general(xy, off, 16, 16, 2, 2, frac_bits=1)


def test_general_points_match_grid(oracle_lib):
    clip = synth.clip(14, 300, 12, n_polygons=10)
    xy = clip.xy.astype(float) / 4
    G, _ = oracle_lib.cfs_grid_general(xy, clip.off, 75, 50, 12, 9, frac_bits=2)
    rng = np.random.default_rng(3)
    k = rng.integers(-12, 13, 40)
    l = rng.integers(-9, 10, 40)
    P = oracle_lib.cfs_points_general(xy, clip.off, 75, 50, k, l, frac_bits=2)
    assert np.array_equal(P, G[k + 12, l + 9])


def _shift_edge(xy, off, e, h):
    """Loops with edge e (joining vertex e to the next of its loop) moved by h
    along its normal: +x for a vertical edge, +y for a horizontal one."""
    xy = np.array(xy, dtype=np.float64)
    m = int(np.searchsorted(off, e, side="right") - 1)
    a, b = e, off[m] + (e - off[m] + 1) % (off[m + 1] - off[m])
    axis = 0 if xy[a, 0] == xy[b, 0] else 1
    xy[a, axis] += h
    xy[b, axis] += h
    return xy


@pytest.mark.parametrize("Nx,Ny,F", [(40, 28, 0), (30, 44, 3)])
def test_general_edge_grad_against_central_differences(oracle_lib, Nx, Ny, F):
    # linear loss Re sum conj(G) F with a fixed random G; both endpoints of an
    # edge move together; step h = 2^-10 keeps the corners on a 2^-12 grid
    clip = synth.clip(31, 400, 6, n_polygons=3)  # larger than the tile: periodic
    Fg = 12
    xy = clip.xy.astype(np.float64) / 2 ** F
    K, L = 6, 5
    rng = np.random.default_rng(4)
    G = rng.normal(size=(2 * K + 1, 2 * L + 1)) + 1j * rng.normal(size=(2 * K + 1, 2 * L + 1))
    g = oracle_lib.edge_grad_general(xy, clip.off, Nx, Ny, K, L, G, frac_bits=F)
    h = 2.0 ** -10
    for e in rng.choice(int(clip.off[-1]), 8, replace=False):
        Fp, _ = oracle_lib.cfs_grid_general(_shift_edge(xy, clip.off, e, h), clip.off, Nx, Ny, K, L,
                                            frac_bits=Fg)
        Fm, _ = oracle_lib.cfs_grid_general(_shift_edge(xy, clip.off, e, -h), clip.off, Nx, Ny,
                                            K, L, frac_bits=Fg)
        fd = float(np.real(np.sum(np.conj(G) * (Fp - Fm)))) / (2 * h)
        assert abs(fd - g[e]) <= 1e-6 * np.max(np.abs(g)) + 1e-9


def test_general_edge_grad_square_tile_matches_square_oracle(oracle_lib):
    clip = synth.clip(32, 64, 6, n_polygons=4)
    rng = np.random.default_rng(6)
    G = rng.normal(size=(13, 11)) + 1j * rng.normal(size=(13, 11))
    g1 = oracle_lib.edge_grad_general(clip.xy.astype(float), clip.off, 64, 64, 6, 5, G)
    g2 = oracle_lib.edge_grad(clip.xy, clip.off, 64, 6, 5, G)
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g2))


@pytest.mark.parametrize("Nx,Ny,F", [(7, 5, 13), (1000, 700, 13), (3000, 2000, 3)])
def test_general_fine_grid_rectangle_closed_form(oracle_lib, Nx, Ny, F):
    # a rectangle with corners on the grid of step 2^-F, periods Nx 2^F up to
    # 2^23 grid units: the coefficients are the product of the two 1-D
    # interval integrals over sqrt(Nx Ny) (the separable closed form)
    rng = np.random.default_rng(F * 1000 + Nx)
    s = 2.0 ** -F
    x0 = rng.integers(0, (Nx << F) // 2) * s
    y0 = rng.integers(0, (Ny << F) // 2) * s
    x1 = x0 + rng.integers(1, (Nx << F) // 3) * s
    y1 = y0 + rng.integers(1, (Ny << F) // 3) * s
    xy = np.array([[x0, y0], [x0, y1], [x1, y1], [x1, y0]])  # clockwise, y up
    off = np.array([0, 4], np.int64)
    K, L = 9, 7
    Fo, area = oracle_lib.cfs_grid_general(xy, off, Nx, Ny, K, L, frac_bits=F)
    G = np.outer(H.rect_interval(x0, x1, np.arange(-K, K + 1), Nx),
                 H.rect_interval(y0, y1, np.arange(-L, L + 1), Ny)) / np.sqrt(Nx * Ny)
    assert area == round((x1 - x0) * (y1 - y0) * 4 ** F)
    assert np.max(np.abs(Fo - G)) <= 1e-9 * abs(G[K, L])
