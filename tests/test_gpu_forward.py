"""GPU parity of the forward transform against the FP64 oracle.

Every case calls the HIP path through the C ABI (via the thin binding) and
compares element by element with the oracle on the same seeded input.
Tolerances (relative to |F[0,0]|, over the whole grid or the sampled set):
FP32 contraction 1e-6, split-bf16 / split-fp16 1e-5; the area and the integer
phases are compared bit for bit.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-6, "bf16": 1e-5, "fp16": 1e-5}


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_5562_amd as P

    torch.cuda.set_device(0)
    return P


def _corners(P, clip):
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    return x, y, s


def _run(P, x, y, s, T, K, L, prec, tile=None):
    F, a = P.forward(x, y, s, T, K, L, precision=prec, tile=tile)
    torch.cuda.synchronize()
    return F.cpu().numpy().astype(np.complex128), int(a.item())


def _err(F, ref, K, L):
    return float(np.max(np.abs(F - ref)) / abs(ref[K, L]))


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_single_polygon_c1(P, oracle_lib, prec):
    clip, _, _ = synth.clip_c1(1)
    _say(f"C1 V={clip.n_vertices} T={clip.T} K={clip.K} prec={prec}")
    ref, area = oracle_lib.cfs_grid(clip.xy, clip.off, clip.T, clip.K, clip.L)
    F, a = _run(P, *_corners(P, clip), clip.T, clip.K, clip.L, prec)
    assert a == area
    assert F[clip.K, clip.L] == np.complex64(np.float32(area / clip.T))
    e = _err(F, ref, clip.K, clip.L)
    _say(f"  err/|F00| = {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5])
def test_tiles_and_ragged_edges(P, oracle_lib, prec, tile):
    # several workgroup tiles in k and l, K != L, a ragged vertex tail; tile
    # variants 3-5 exist for the split forms only
    if prec == "fp32" and tile >= 3:
        pytest.skip("split-only tile variant")
    T, K, L = 1024, 150, 97
    clip = synth.clip(31, T, K, L, n_polygons=211)
    _say(f"ragged V={clip.n_vertices} T={T} K={K} L={L} prec={prec} tile={tile}")
    ref, area = oracle_lib.cfs_grid(clip.xy, clip.off, T, K, L)
    F, a = _run(P, *_corners(P, clip), T, K, L, prec, tile=tile)
    assert a == area
    e = _err(F, ref, K, L)
    _say(f"  err/|F00| = {e:.3e}")
    assert e <= TOL[prec]


def test_phases_bit_exact(P):
    clip = synth.clip(8, 4096, 255, n_polygons=300)
    x, y, s = _corners(P, clip)
    # include negative and out-of-tile coordinates
    x = x.astype(np.int64) - 5000
    y = y.astype(np.int64) + 9000
    for T in (4096, 64, 8192):
        for axis, c in ((0, x), (1, y)):
            p = P.debug_phases(x.astype(np.int32), y.astype(np.int32), s, T, 1, 300, axis=axis)
            got = p.cpu().numpy().astype(np.int64)
            want = (np.arange(1, 301)[:, None] * c[None, :]) % T
            assert np.array_equal(got, want)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("tile", [None, 0])  # None: direct form at this size; 0: staged MFMA path
def test_degenerate_sizes(P, oracle_lib, prec, tile):
    clip = synth.clip(12, 512, 20, n_polygons=9)
    x, y, s = _corners(P, clip)
    for K, L in ((0, 0), (0, 7), (9, 0), (1, 1), (33, 2)):
        _say(f"degenerate K={K} L={L} prec={prec} tile={tile}")
        ref, area = oracle_lib.cfs_grid(clip.xy, clip.off, 512, K, L)
        F, a = _run(P, x, y, s, 512, K, L, prec, tile=tile)
        assert a == area
        assert _err(F, ref, K, L) <= TOL[prec]
    # no corners at all: every coefficient is zero
    e = np.zeros(0, np.int32)
    F, a = _run(P, e, e, e.astype(np.int8), 512, 5, 4, prec, tile=tile)
    assert a == 0 and np.all(F == 0)


def _launches(P, fn):
    h = P.default_handle()
    h.profile_begin(("direct", "contract"))
    fn()
    prof = h.profile_end()
    return prof["direct"][1], prof["contract"][1]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_direct_form_small_problems(P, oracle_lib, prec):
    # At most 1024 corners and 2^22 corner-coefficient pairs: one launch of
    # the FP64 direct form whatever the precision (so the FP32 bound holds);
    # a forced tile variant runs the staged MFMA path on the same input.
    c1, _, _ = synth.clip_c1(1)
    big = synth.clip(41, 4096, 20, n_polygons=60)
    out = synth.clip(42, 300, 12, n_polygons=25)
    cases = [(c1.xy, c1.off, c1.T, c1.K, c1.L),
             (big.xy, big.off, 4096, 20, 20),
             (synth.shift_loops(out.xy, -150, 77), out.off, 2, 6, 6),        # K > T
             (synth.shift_loops(out.xy, 70000, -90000), out.off, 512, 40, 9)]
    for xy, off, T, K, L in cases:
        x, y, s, _, _ = P.loops_to_corners(xy, off)
        V = x.size
        assert V <= 1024 and V * (K + 1) * (2 * L + 1) <= 1 << 22
        ref, area = oracle_lib.cfs_grid(xy, off, T, K, L)
        res = {}
        for tile in (None, 0):
            def go():
                res[tile] = _run(P, x, y, s, T, K, L, prec, tile=tile)
            nd, nc = _launches(P, go)
            assert (nd, nc) == ((1, 0) if tile is None else (0, 1 if K and L else 0))
            F, a = res[tile]
            assert a == area
            e = _err(F, ref, K, L)
            _say(f"small V={V} T={T} K={K} L={L} {prec} tile={tile}: err/|F00| = {e:.3e}")
            assert e <= (TOL["fp32"] if tile is None else TOL[prec])
        assert res[None][0][K, L] == res[0][0][K, L]  # the same exact DC entry


def test_direct_form_threshold(P):
    # one step past either bound (1024 corners, 2^22 corner-coefficient
    # pairs) selects the staged path
    clip = synth.clip(43, 2048, 8, n_polygons=50)
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    V = x.size
    assert 512 < V <= 1024
    lo = max(l for l in range(4096) if V * 2 * (2 * l + 1) <= 1 << 22)  # K = 1
    for l, want in ((lo, (1, 0)), (lo + 1, (0, 1))):
        assert _launches(P, lambda: _run(P, x, y, s, 2048, 1, l, "bf16")) == want
    many = synth.clip(44, 2048, 8, n_polygons=70)
    xm, ym, sm, _, _ = P.loops_to_corners(many.xy, many.off)
    assert xm.size > 1024
    assert _launches(P, lambda: _run(P, xm, ym, sm, 2048, 1, 1, "bf16")) == (0, 1)


@pytest.mark.parametrize("T", [2, 16, 8192])
def test_periods_and_out_of_tile(P, oracle_lib, T):
    # coordinates beyond [0, T) and negative: the CFS of the periodisation
    clip = synth.clip(13, 300, 12, n_polygons=25)
    xy = synth.shift_loops(clip.xy, -150, 77)
    K = min(12, 3 * T)
    ref, area = oracle_lib.cfs_grid(xy, clip.off, T, K, K)
    x, y, s, _, _ = P.loops_to_corners(xy, clip.off)
    for prec in ("fp32", "fp16"):
        F, a = _run(P, x, y, s, T, K, K, prec)
        assert a == area
        assert _err(F, ref, K, K) <= TOL[prec]


def test_deterministic_and_hermitian(P):
    clip = synth.clip(14, 2048, 127, n_polygons=400)
    x, y, s = _corners(P, clip)
    F1, _ = _run(P, x, y, s, 2048, 127, 127, "bf16")
    F2, _ = _run(P, x, y, s, 2048, 127, 127, "bf16")
    assert np.array_equal(F1, F2)
    assert np.array_equal(F1, np.conj(F1[::-1, ::-1]))


def _sample_points(K, L, n, seed):
    rng = np.random.default_rng(seed)
    lo = [(k, l) for k in range(-8, 9) for l in range(-8, 9)]
    kk = np.concatenate([np.array([p[0] for p in lo]), rng.integers(-K, K + 1, n)])
    ll = np.concatenate([np.array([p[1] for p in lo]), rng.integers(-L, L + 1, n)])
    return kk, ll


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_full_size_layout_clip_sampled(P, oracle_lib, prec):
    # 2,000 polygons, T = 4096, |k|,|l| <= 255 (the layout-clip workload)
    T, K = 4096, 255
    clip = synth.clip(2, T, K, n_polygons=2000)
    _say(f"layout clip V={clip.n_vertices} T={T} K={K} prec={prec}")
    kk, ll = _sample_points(K, K, 400, 1)
    ref = oracle_lib.cfs_points(clip.xy, clip.off, T, kk, ll)
    F, a = _run(P, *_corners(P, clip), T, K, K, prec)
    f00 = oracle_lib.cfs_points(clip.xy, clip.off, T, [0], [0])[0]
    e = float(np.max(np.abs(F[kk + K, ll + K] - ref)) / abs(f00))
    _say(f"  err/|F00| = {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_full_size_precision_clip_sampled(P, oracle_lib, prec):
    # 200k corners, T = 8192, |k|,|l| <= 511 (the precision-form workload)
    T, K = 8192, 511
    clip = synth.clip(3, T, K, min_vertices=200_000)
    _say(f"precision clip V={clip.n_vertices} T={T} K={K} prec={prec}")
    kk, ll = _sample_points(K, K, 300, 2)
    ref = oracle_lib.cfs_points(clip.xy, clip.off, T, kk, ll)
    f00 = oracle_lib.cfs_points(clip.xy, clip.off, T, [0], [0])[0]
    F, a = _run(P, *_corners(P, clip), T, K, K, prec)
    e = float(np.max(np.abs(F[kk + K, ll + K] - ref)) / abs(f00))
    _say(f"  err/|F00| = {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_disjoint_low_fill_clip(P, oracle_lib, prec):
    # polygons confined to disjoint cells (fill factor well below one, as in a
    # real layer): the hardest case for an error bound relative to |F[0,0]|
    T, K = 8192, 511
    clip = synth.clip(33, T, K, min_vertices=200_000, disjoint=True)
    _say(f"disjoint clip V={clip.n_vertices} T={T} K={K} prec={prec}")
    kk, ll = _sample_points(K, K, 300, 3)
    ref = oracle_lib.cfs_points(clip.xy, clip.off, T, kk, ll)
    f00 = oracle_lib.cfs_points(clip.xy, clip.off, T, [0], [0])[0]
    F, a = _run(P, *_corners(P, clip), T, K, K, prec)
    e = float(np.max(np.abs(F[kk + K, ll + K] - ref)) / abs(f00))
    _say(f"  fill {abs(f00) * T / T**2:.3f}, err/|F00| = {e:.3e}")
    assert e <= TOL[prec]


def _hyperbola_points(K, L, kl_max):
    # every (k, l) with k, l != 0 and |k l| <= kl_max inside the grid: where
    # the 1/(k l) factor of alpha amplifies the contraction's rounding most
    pts = [(k, l) for k in range(-K, K + 1) for l in range(-L, L + 1)
           if k and l and abs(k * l) <= kl_max]
    a = np.array(pts)
    return a[:, 0], a[:, 1]


@pytest.mark.parametrize("case", ["layout", "precision"])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_disjoint_low_fill_near_axes(P, oracle_lib, prec, case):
    # low-fill clips checked on every coefficient with |k l| <= 160 (both
    # strips next to the axes and the low corner), against the bound 1e-5
    # |F[0,0]| of the split forms: the guard region has to widen here
    if case == "layout":
        T, K = 4096, 255
        clip = synth.clip(22, T, K, n_polygons=2000, disjoint=True)
    else:
        T, K = 8192, 511
        clip = synth.clip(33, T, K, min_vertices=200_000, disjoint=True)
    kk, ll = _hyperbola_points(K, K, 160)
    _say(f"disjoint {case} clip V={clip.n_vertices} T={T} K={K} prec={prec}, {kk.size} points")
    ref = oracle_lib.cfs_points(clip.xy, clip.off, T, kk, ll)
    f00 = oracle_lib.cfs_points(clip.xy, clip.off, T, [0], [0])[0]
    F, a = _run(P, *_corners(P, clip), T, K, K, prec)
    err = np.abs(F[kk + K, ll + K] - ref) / abs(f00)
    w = int(np.argmax(err))
    _say(f"  fill {abs(f00) * T / T**2:.3f}, max err/|F00| = {err[w]:.3e} at ({kk[w]},{ll[w]})")
    assert err[w] <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_band_forward(P, oracle_lib, prec):
    # low-pass forward: |k| <= kmax, |l| <= lmax, optionally k^2 + l^2 <= r^2;
    # the rest of the (2K+1)(2L+1) grid is zero
    T, K, L = 1024, 150, 97
    clip = synth.clip(31, T, K, L, n_polygons=211)
    x, y, s = _corners(P, clip)
    ref, _ = oracle_lib.cfs_grid(clip.xy, clip.off, T, K, L)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-L, L + 1), indexing="ij")
    for band, radius in (((40, 70), None), ((K, L), 35.5), ((20, 60), 50.0), ((0, 30), None)):
        _say(f"band {band} radius {radius} prec={prec}")
        F, a = P.forward(x, y, s, T, K, L, precision=prec, band=band, radius=radius)
        torch.cuda.synchronize()
        F = F.cpu().numpy().astype(np.complex128)
        inside = (np.abs(kk) <= band[0]) & (np.abs(ll) <= band[1])
        if radius is not None:
            inside &= kk ** 2 + ll ** 2 <= radius ** 2
        assert np.all(F[~inside] == 0)
        e = float(np.max(np.abs(F[inside] - ref[inside])) / abs(ref[K, L]))
        _say(f"  err/|F00| = {e:.3e}")
        assert e <= TOL[prec]


def test_band_forward_skips_tiles_full_size(P, oracle_lib):
    # precision clip with a disc of radius 200: the tiles beyond it are skipped
    T, K = 8192, 511
    clip = synth.clip(3, T, K, min_vertices=200_000)
    x, y, s = _corners(P, clip)
    r = 200.0
    F, _ = P.forward(x, y, s, T, K, K, precision="bf16", radius=r)
    torch.cuda.synchronize()
    F = F.cpu().numpy()
    kk, ll = _sample_points(K, K, 300, 4)
    inside = kk ** 2 + ll ** 2 <= r * r
    ref = oracle_lib.cfs_points(clip.xy, clip.off, T, kk[inside], ll[inside])
    f00 = oracle_lib.cfs_points(clip.xy, clip.off, T, [0], [0])[0]
    e = float(np.max(np.abs(F[kk[inside] + K, ll[inside] + K] - ref)) / abs(f00))
    _say(f"disc r={r}: {int(inside.sum())} points inside, err/|F00| = {e:.3e}")
    assert e <= TOL["bf16"]
    assert np.all(F[kk[~inside] + K, ll[~inside] + K] == 0)
    k2, l2 = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    assert np.all(F[k2 ** 2 + l2 ** 2 > r * r] == 0)
