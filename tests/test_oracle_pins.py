"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

The paper prints no FCFS coefficient values, so every pin is mathematical:
closed forms, exact integer identities, brute force on tiny inputs and
symmetries.  Each one is chosen so that a plausible slip in the oracle (a
dropped axis term, a wrong sign in alpha_{k,l}, swapped k and l, a wrong
orientation rule, a phase reduced the wrong way) breaks at least one of them.
"""
import numpy as np
import pytest

import synth
from tests import helpers as H


def _rect_loop(x1, y1, x2, y2):
    return synth.rectangle_loop(x1, y1, x2, y2), np.array([0, 4])


# Both full-grid forms of the oracle take every pin below: the C edge sums
# (cfs_grid) and the numpy form whose general term is one matrix product
# (cfs_grid_matmul, used for full grids of large clips).
@pytest.fixture(params=["edge_sums", "matmul"])
def grid(request, oracle_lib):
    if request.param == "edge_sums":
        return lambda xy, off, T, K, L: oracle_lib.cfs_grid(xy, off, T, K, L)
    return lambda xy, off, T, K, L: oracle_lib.cfs_grid_matmul(xy, off, T, K, L)


@pytest.mark.parametrize("form", ["lattice", "real", "matmul"])
def test_single_rectangle_sinc_product(oracle_lib, form):
    # Sec. II-C basis integrated over [x1,x2) x [y1,y2): sinc product, all
    # (k, l) including the axes and DC.  dx != dy and K != L catch a k/l swap.
    T, K, L = 64, 11, 7
    x1, y1, x2, y2 = 3, 5, 20, 41
    xy, off = _rect_loop(x1, y1, x2, y2)
    lattice = form != "real"
    if form == "matmul":
        F, area = oracle_lib.cfs_grid_matmul(xy, off, T, K, L)
    else:
        F, area = oracle_lib.cfs_grid(xy, off, T, K, L, lattice=lattice)
    G = H.rect_cfs(x1, y1, x2, y2, T, K, L)
    assert np.max(np.abs(F - G)) <= 1e-13 * abs(G[K, L])
    if lattice:
        assert area == (x2 - x1) * (y2 - y1)


def test_rectangle_counter_clockwise_is_reversed(grid):
    # Clockwise order is the paper's convention (Sec. II-A2); the reversed loop
    # describes the same set and must give the same coefficients.
    T, K = 32, 6
    xy, off = _rect_loop(2, 3, 9, 17)
    F1, a1 = grid(xy, off, T, K, K)
    F2, a2 = grid(xy[::-1].copy(), off, T, K, K)
    assert a1 == a2 == 7 * 14
    assert np.max(np.abs(F1 - F2)) <= 1e-14


def _union_clip(seed, T, n_polys, lo=3, hi=12):
    rng = np.random.default_rng(seed)
    loops, rects_all = [], []
    while len(loops) < n_polys:
        n = int(rng.integers(1, 5))
        r = []
        for _ in range(n):
            x1 = int(rng.integers(0, T - hi))
            y1 = int(rng.integers(0, T - hi))
            r.append((x1, y1, x1 + int(rng.integers(lo, hi)), y1 + int(rng.integers(lo, hi))))
        lp = synth.loops_of_rect_union(r)
        if lp is None or len(lp) != 1:
            continue
        loops.append(lp[0])
        rects_all.append(r)
    off = np.zeros(len(loops) + 1, np.int64)
    off[1:] = np.cumsum([p.shape[0] for p in loops])
    return np.concatenate(loops), off, rects_all


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_raster_identity(grid, seed):
    # Lattice polygons are unions of unit cells; each cell's CFS is a closed
    # form, so the sum over the rasterised cells is an exact brute force.
    # Overlapping polygons add (signal model, Sec. III-A).
    T, K, L = 48, 13, 9
    xy, off, _ = _union_clip(seed, T, 4)
    F, area = grid(xy, off, T, K, L)
    img = H.raster(xy, off, T)
    R = H.raster_cfs(img, T, K, L)
    assert area == int(img.sum())
    assert np.max(np.abs(F - R)) <= 1e-12 * abs(R[K, L])


def test_fft_of_corner_image(grid):
    # Step 4 of Sec. III-C1: the double sum is a 2-D DFT of the sparse +/-1
    # corner image.  The corner weights come from the raster (mixed second
    # difference), not from the oracle's edge walk.
    T, K, L = 64, 20, 17
    xy, off, _ = _union_clip(7, T, 3)
    F, _ = grid(xy, off, T, K, L)
    W = H.corner_image(H.raster(xy, off, T))
    # corners on x = T or y = T wrap to 0 under the period
    D = np.fft.fft2(_fold(W, T))
    k = np.arange(-K, K + 1)
    l = np.arange(-L, L + 1)
    S = D[np.ix_(k % T, l % T)]
    kk, ll = np.meshgrid(k, l, indexing="ij")
    with np.errstate(divide="ignore", invalid="ignore"):
        Fk = -T / (4 * np.pi**2 * kk * ll) * S
    m = (kk != 0) & (ll != 0)
    assert np.max(np.abs(F[m] - Fk[m])) <= 1e-12 * abs(F[K, L])
    # and the raw corner sum vanishes on the axes (telescoping, Lemma 1)
    assert np.max(np.abs(S[K, :])) <= 1e-9 and np.max(np.abs(S[:, L])) <= 1e-9


def _fold(W, T):
    out = np.zeros((T, T), dtype=np.float64)
    for i in range(W.shape[0]):
        for j in range(W.shape[1]):
            if W[i, j]:
                out[i % T, j % T] += W[i, j]
    return out


def test_area_matches_shoelace_and_dc(oracle_lib):
    clip = synth.clip(11, 4096, 0, n_polygons=50)
    areas = oracle_lib.loop_areas(clip.xy, clip.off)
    # clockwise (y up) loops have negative shoelace sum in the usual sense
    assert np.array_equal(areas, -H.shoelace2(clip.xy, clip.off) // 2)
    assert np.all(areas > 0)
    F, A = oracle_lib.cfs_grid(clip.xy, clip.off, 4096, 0, 0)
    assert A == int(areas.sum())
    assert F[0, 0].real == pytest.approx(A / 4096, rel=1e-15)
    Fm, Am = oracle_lib.cfs_grid_matmul(clip.xy, clip.off, 4096, 0, 0)
    assert Am == A and Fm[0, 0] == F[0, 0]


def test_linearity_and_inclusion_exclusion(grid):
    # Sec. III-A linearity: f(A u B) = f(A) + f(B) - f(A n B).
    T, K, L = 128, 9, 12
    a = (10, 20, 70, 60)
    b = (40, 35, 100, 90)
    inter = (40, 35, 70, 60)
    u = synth.loops_of_rect_union([a, b])
    assert u is not None and len(u) == 1
    Fu, Au = grid(u[0], [0, u[0].shape[0]], T, K, L)
    Fa, Aa = grid(*_rect_loop(*a), T, K, L)
    Fb, Ab = grid(*_rect_loop(*b), T, K, L)
    Fi, Ai = grid(*_rect_loop(*inter), T, K, L)
    assert Au == Aa + Ab - Ai
    assert np.max(np.abs(Fu - (Fa + Fb - Fi))) <= 1e-12 * abs(Fu[K, L])
    # several loops in one call add up
    both = np.concatenate([synth.rectangle_loop(*a), synth.rectangle_loop(*b)])
    F2, A2 = grid(both, [0, 4, 8], T, K, L)
    assert A2 == Aa + Ab
    assert np.max(np.abs(F2 - (Fa + Fb))) <= 1e-12 * abs(F2[K, L])


def test_symmetries(grid):
    T, K, L = 256, 12, 10
    xy, off, _ = _union_clip(3, 200, 5, lo=10, hi=40)
    F, _ = grid(xy, off, T, K, L)
    # Hermitian: F[-k,-l] = conj F[k,l] (real signal)
    assert np.max(np.abs(F - np.conj(F[::-1, ::-1]))) <= 1e-13 * abs(F[K, L])
    # shift theorem, axes and DC included
    dx, dy = 17, -5
    Fs, _ = grid(synth.shift_loops(xy, dx, dy), off, T, K, L)
    k = np.arange(-K, K + 1)[:, None]
    l = np.arange(-L, L + 1)[None, :]
    ph = np.exp(-2j * np.pi * (k * dx + l * dy) / T)
    assert np.max(np.abs(Fs - F * ph)) <= 1e-12 * abs(F[K, L])
    # translation by whole periods changes nothing (exact integer reduction)
    Ft, _ = grid(synth.shift_loops(xy, 3 * T, -2 * T), off, T, K, L)
    assert np.max(np.abs(Ft - F)) <= 1e-12 * abs(F[K, L])
    # integer scaling by m with period m T multiplies F by m
    m = 3
    Fm, _ = grid(xy * m, off, m * T, K, L)
    assert np.max(np.abs(Fm - m * F)) <= 1e-12 * abs(Fm[K, L])
    # rotation by +90 degrees, (x, y) -> (-y, x): F'[k, l] = F[l, -k]
    rot = np.stack([-xy[:, 1], xy[:, 0]], axis=1)
    Fr, _ = grid(rot, off, T, L, K)
    # Fr is indexed [k + L, l + K]; F[l, -k] is F[l + K, -k + L]
    assert np.max(np.abs(Fr - F.T[::-1, :])) <= 1e-12 * abs(F[K, L])


def test_points_match_grid(oracle_lib):
    T, K = 512, 15
    clip = synth.clip(5, T, K, n_polygons=20)
    F, _ = oracle_lib.cfs_grid(clip.xy, clip.off, T, K, K)
    rng = np.random.default_rng(0)
    kk = rng.integers(-K, K + 1, 40)
    ll = rng.integers(-K, K + 1, 40)
    P = oracle_lib.cfs_points(clip.xy, clip.off, T, kk, ll)
    assert np.array_equal(P, F[kk + K, ll + K])


def test_rejects_invalid_loops(oracle_lib):
    bad = [
        (np.array([[0, 0], [0, 5], [5, 5]]), [0, 3]),                 # odd count
        (np.array([[0, 0], [0, 5], [5, 6], [5, 0]]), [0, 4]),         # slanted edge
        (np.array([[0, 0], [0, 5], [0, 9], [5, 9], [5, 0], [3, 0]]), [0, 6]),  # no alternation
    ]
    for xy, off in bad:
        with pytest.raises(oracle_lib.OracleError):
            oracle_lib.cfs_grid(xy, off, 16, 2, 2)
        with pytest.raises(oracle_lib.EdgeFormError):
            oracle_lib.cfs_grid_matmul(xy, off, 16, 2, 2)


def test_matmul_form_matches_edge_sums_on_a_clip(oracle_lib):
    # the two forms on a layout-like clip, K != L, polygons sticking out of
    # the tile (phases reduced modulo T, moments from the raw coordinates)
    T, K, L = 512, 21, 14
    clip = synth.clip(9, 600, K, L, n_polygons=30)
    F, A = oracle_lib.cfs_grid(clip.xy, clip.off, T, K, L)
    G, B = oracle_lib.cfs_grid_matmul(clip.xy, clip.off, T, K, L)
    assert A == B
    assert np.max(np.abs(F - G)) <= 1e-13 * abs(F[K, L])


def test_gradient_rectangle_closed_form(oracle_lib):
    # d/dx2 of the rectangle integral is e(k x2) times the y integral
    # (fundamental theorem of calculus), for every (k, l) including the axes.
    T, K, L = 64, 9, 6
    x1, y1, x2, y2 = 4, 7, 29, 22
    xy, off = _rect_loop(x1, y1, x2, y2)
    rng = np.random.default_rng(3)
    G = rng.normal(size=(2 * K + 1, 2 * L + 1)) + 1j * rng.normal(size=(2 * K + 1, 2 * L + 1))
    g = oracle_lib.edge_grad(xy, off, T, K, L, G)
    k = np.arange(-K, K + 1)
    l = np.arange(-L, L + 1)
    e = lambda f, t: np.exp(-2j * np.pi * f * t / T)  # noqa: E731
    Ix = H.rect_interval(x1, x2, k, T)[:, None]
    Iy = H.rect_interval(y1, y2, l, T)[None, :]
    dF = {
        0: -e(k, x1)[:, None] * Iy / T,   # vertical edge at x1 moves along +x
        1: Ix * e(l, y2)[None, :] / T,    # horizontal edge at y2 moves along +y
        2: e(k, x2)[:, None] * Iy / T,
        3: -Ix * e(l, y1)[None, :] / T,
    }
    for i in range(4):
        want = np.real(np.sum(np.conj(G) * dF[i]))
        assert g[i] == pytest.approx(want, rel=1e-11, abs=1e-12)


def test_gradient_matches_central_differences(oracle_lib):
    # Real-coordinate mode; a loss with a circular pupil, as in the
    # differentiation form.  Step 1e-3 (central differences).
    T, K, L = 64, 20, 17
    xy, off, _ = _union_clip(4, 60, 2, lo=8, hi=25)
    xy = xy.astype(np.float64)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-L, L + 1), indexing="ij")
    Hp = (kk**2 + ll**2 <= (0.35 * K) ** 2).astype(np.float64)
    rng = np.random.default_rng(1)
    Gt = Hp * (rng.normal(size=Hp.shape) + 1j * rng.normal(size=Hp.shape)) * 1e-2

    def loss(p):
        F, _ = oracle_lib.cfs_grid(p, off, T, K, L, lattice=False)
        return float(np.sum(np.abs(Hp * F - Gt) ** 2))

    F0, _ = oracle_lib.cfs_grid(xy, off, T, K, L, lattice=False)
    Gc = 2 * Hp * (Hp * F0 - Gt)  # dLoss/dRe F + j dLoss/dIm F
    g = oracle_lib.edge_grad(xy, off, T, K, L, Gc, lattice=False)
    gl = oracle_lib.edge_grad(xy, off, T, K, L, Gc, lattice=True)
    assert np.max(np.abs(g - gl)) <= 1e-12 * np.max(np.abs(g))
    h = 1e-3
    n = int(off[-1])
    fd = np.zeros(n)
    for e in range(n):
        a = e
        b = off[np.searchsorted(off, e, side="right") - 1] + (
            (e - off[np.searchsorted(off, e, side="right") - 1] + 1)
            % (off[np.searchsorted(off, e, side="right")] - off[np.searchsorted(off, e, side="right") - 1]))
        axis = 1 if xy[a, 1] == xy[b, 1] else 0  # horizontal edges move in y
        p1 = xy.copy()
        p2 = xy.copy()
        p1[[a, b], axis] += h
        p2[[a, b], axis] -= h
        fd[e] = (loss(p1) - loss(p2)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * np.max(np.abs(g))
