"""GPU parity of the general-tile forward transform (fcfs_forward_general:
periods Nx != Ny, not powers of two, corners on a 2^-F grid) against the
general-tile oracle.

Tolerances as for the square tile: FP32 1e-6 |F[0,0]|, split 1e-5 |F[0,0]|;
the area (sum s x y in grid units) is exact."""
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


def _say(msg):
    print(msg, flush=True)


def _gpu(P, xy, off, Nx, Ny, K, L, F, prec):
    x, y, s, _, _ = P.loops_to_corners(xy, off)
    Fg, a = P.forward_general(x, y, s, Nx, Ny, K, L, frac_bits=F, precision=prec)
    torch.cuda.synchronize()
    return Fg.cpu().numpy().astype(np.complex128), int(a.item())


@pytest.mark.parametrize("Nx,Ny,F,K,L,npol,seed", [
    (3000, 2000, 0, 40, 33, 150, 21),     # non-square, not powers of two
    (750, 1000, 2, 37, 45, 150, 22),      # quarter-unit grid: periods 3000 x 4000
    (1000, 1000, 0, 70, 70, 200, 23),     # equal periods (one shared table)
    (7, 5, 3, 30, 29, 6, 24),             # tiny odd tile, frequencies past the period
    (2048, 1536, 1, 3, 0, 60, 25),        # L = 0: axes only
])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_general_full_grid(P, oracle_lib, Nx, Ny, F, K, L, npol, seed, prec):
    Mx, My = Nx << F, Ny << F
    clip = synth.clip(seed, max(Mx, My), K, L, n_polygons=npol)  # grid units
    xy = clip.xy.astype(np.float64) / 2 ** F
    ref, area = oracle_lib.cfs_grid_general(xy, clip.off, Nx, Ny, K, L, frac_bits=F)
    Fg, a = _gpu(P, clip.xy, clip.off, Nx, Ny, K, L, F, prec)
    assert a == area
    e = float(np.max(np.abs(Fg - ref)) / abs(ref[K, L]))
    _say(f"general {Nx}x{Ny} F={F} K={K} L={L} {prec}: err/|F00| = {e:.3e}")
    assert e <= TOL[prec]


def test_general_negative_and_outside_coordinates(P, oracle_lib):
    clip = synth.clip(26, 900, 20, n_polygons=40)
    xy = synth.shift_loops(clip.xy, -523, 1777)
    ref, area = oracle_lib.cfs_grid_general(xy.astype(float) / 2, clip.off, 450, 300, 20, 18,
                                           frac_bits=1)
    for prec in ("fp32", "bf16"):
        Fg, a = _gpu(P, xy, clip.off, 450, 300, 20, 18, 1, prec)
        assert a == area
        assert float(np.max(np.abs(Fg - ref)) / abs(ref[20, 18])) <= TOL[prec]


def test_general_square_power_of_two_matches_fast_path(P, oracle_lib):
    clip = synth.clip(27, 1024, 100, n_polygons=300)
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    ref, _ = oracle_lib.cfs_grid(clip.xy, clip.off, 1024, 100, 100)
    for prec in ("fp32", "bf16"):
        Fg, _ = P.forward_general(x, y, s, 1024, 1024, 100, 100, precision=prec)
        Ff, _ = P.forward(x, y, s, 1024, 100, 100, precision=prec)
        torch.cuda.synchronize()
        for F_ in (Fg, Ff):
            e = float(np.max(np.abs(F_.cpu().numpy().astype(np.complex128) - ref)) / abs(ref[100, 100]))
            assert e <= TOL[prec]


def test_general_layout_clip_sampled(P, oracle_lib):
    # 2,000 polygons on a 4000 x 3000 tile with half-unit corners (periods
    # 8000 x 6000 in grid units), |k|, |l| <= 255: sampled coefficients
    Nx, Ny, F, K = 4000, 3000, 1, 255
    clip = synth.clip(2, 8000, K, n_polygons=2000)
    xy = clip.xy.astype(np.float64) / 2
    rng = np.random.default_rng(8)
    lo = np.array([(k, l) for k in range(-8, 9) for l in range(-8, 9)])
    kk = np.concatenate([lo[:, 0], rng.integers(-K, K + 1, 300)])
    ll = np.concatenate([lo[:, 1], rng.integers(-K, K + 1, 300)])
    ref = oracle_lib.cfs_points_general(xy, clip.off, Nx, Ny, kk, ll, frac_bits=F)
    f00 = abs(oracle_lib.cfs_points_general(xy, clip.off, Nx, Ny, [0], [0], frac_bits=F)[0])
    for prec in ("fp32", "bf16"):
        Fg, _ = _gpu(P, clip.xy, clip.off, Nx, Ny, K, K, F, prec)
        e = float(np.max(np.abs(Fg[kk + K, ll + K] - ref)) / f00)
        _say(f"general layout clip {prec}: err/|F00| = {e:.3e} over {kk.size} points")
        assert e <= TOL[prec]


def test_general_empty_and_errors(P):
    e = np.zeros(0, np.int32)
    Fg, a = P.forward_general(e, e, e.astype(np.int8), 300, 200, 5, 4)
    torch.cuda.synchronize()
    assert int(a.item()) == 0 and bool((Fg == 0).all())
    sq = synth.rectangle_loop(0, 0, 3, 3)
    x, y, s, _, _ = P.loops_to_corners(sq, np.array([0, 4]))
    # periods past 2^24 grid units, F > 13 and a period below 2
    for Nx, Ny, F in ((5000, 100, 12), (100, 100, 14), (100, 2049, 13), (1, 1, 0)):
        with pytest.raises(P.FcfsError):
            P.forward_general(x, y, s, Nx, Ny, 4, 4, frac_bits=F)


# ---------------------------------------------------------------- adjoint
GTOL = {"fp32": 1e-5, "bf16": 1e-4, "fp16": 1e-4}


def _rand_G(K, L, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(2 * K + 1, 2 * L + 1)) + 1j * rng.normal(size=(2 * K + 1, 2 * L + 1))


@pytest.mark.parametrize("Nx,Ny,F,K,L,seed", [
    (3000, 2000, 0, 37, 70, 51),      # several GEMM column groups, K != L
    (750, 1000, 2, 40, 33, 52),       # quarter-unit grid, periods 3000 x 4000
    (8192, 8000, 0, 20, 20, 53),      # both tables at their largest (LDS full)
])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_general_adjoint_random_cotangent(P, oracle_lib, Nx, Ny, F, K, L, seed, prec):
    Mx, My = Nx << F, Ny << F
    clip = synth.clip(seed, max(Mx, My), K, L, n_polygons=40)
    xy = clip.xy.astype(np.float64) / 2 ** F
    G = _rand_G(K, L, seed)
    want = oracle_lib.edge_grad_general(xy, clip.off, Nx, Ny, K, L, G.astype(np.complex64),
                                        frac_bits=F)
    x, y, s, he, ve = P.loops_to_corners(clip.xy, clip.off)
    Gd = torch.as_tensor(G.astype(np.complex64)).cuda()
    gx, gy = P.adjoint_general(x, y, s, Nx, Ny, K, L, Gd, frac_bits=F, precision=prec)
    got = P.edge_grad(gx, gy, he, ve, x.size).cpu().numpy().astype(np.float64)
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    _say(f"general adjoint {Nx}x{Ny} F={F} {prec}: err/max|g| = {e:.3e}")
    assert e <= GTOL[prec]


def test_general_adjoint_band_and_disc(P, oracle_lib):
    Nx, Ny, F, K, L = 1500, 1100, 1, 48, 48
    clip = synth.clip(54, 3000, K, L, n_polygons=60)
    xy = clip.xy.astype(np.float64) / 2
    G = _rand_G(K, L, 5)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-L, L + 1), indexing="ij")
    G[(kk ** 2 + ll ** 2) > 17.5 ** 2] = 0
    want = oracle_lib.edge_grad_general(xy, clip.off, Nx, Ny, K, L, G.astype(np.complex64),
                                        frac_bits=F)
    x, y, s, he, ve = P.loops_to_corners(clip.xy, clip.off)
    Gd = torch.as_tensor(G.astype(np.complex64)).cuda()
    gx, gy = P.adjoint_general(x, y, s, Nx, Ny, K, L, Gd, frac_bits=F, precision="fp32",
                               band=(20, 20), radius=17.5)
    got = P.edge_grad(gx, gy, he, ve, x.size).cpu().numpy().astype(np.float64)
    assert float(np.max(np.abs(got - want)) / np.max(np.abs(want))) <= GTOL["fp32"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_general_autograd_fractional_offsets(P, oracle_lib, prec):
    # edges moved by multiples of a quarter unit on a 600 x 420 tile; loss
    # sum |F|^2: forward against the oracle at the moved corners, gradient
    # against the oracle's analytic gradient there (cotangent 2 F)
    Nx, Ny, F, K = 600, 420, 2, 24
    clip = synth.clip(55, 420, K, n_polygons=12)
    geom = P.Geometry(clip.xy, clip.off, Nx, K, Ny=Ny, frac_bits=F)
    rng = np.random.default_rng(9)
    offs = rng.integers(-3, 4, geom.n_edges) / 4.0
    off = torch.tensor(offs, dtype=torch.float32, device="cuda", requires_grad=True)
    Fv = P.FCFSFunction.apply(off, geom, prec)
    (Fv.abs() ** 2).sum().backward()
    torch.cuda.synchronize()
    # the moved loops (true units) for the oracle
    xy = clip.xy.astype(np.float64).copy()
    for m in range(clip.off.size - 1):
        a0, a1 = clip.off[m], clip.off[m + 1]
        for e in range(a0, a1):
            b = a0 + (e - a0 + 1) % (a1 - a0)
            axis = 0 if clip.xy[e, 0] == clip.xy[b, 0] else 1
            xy[e, axis] += offs[e]
            xy[b, axis] += offs[e]
    ref, _ = oracle_lib.cfs_grid_general(xy, clip.off, Nx, Ny, K, K, frac_bits=F)
    Fg = Fv.detach().cpu().numpy().astype(np.complex128)
    assert float(np.max(np.abs(Fg - ref)) / abs(ref[K, K])) <= TOL[prec]
    want = oracle_lib.edge_grad_general(xy, clip.off, Nx, Ny, K, K, 2 * ref, frac_bits=F)
    got = off.grad.cpu().numpy().astype(np.float64)
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    _say(f"general autograd {prec}: err/max|g| = {e:.3e}")
    assert e <= GTOL[prec]


# ---------------------------------------------------------------- low-pass
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_general_band_forward(P, oracle_lib, prec):
    # band |k| <= 60, |l| <= 40 and disc k^2 + l^2 <= 45^2 of a 1500 x 1100
    # tile on half units (periods 3000 x 2200): the oracle's full grid inside,
    # exact zeros outside; tiles of 128 x 128 frequencies beyond the disc skipped
    Nx, Ny, F, K, L = 1500, 1100, 1, 300, 140
    clip = synth.clip(56, 3000, K, L, n_polygons=80)
    xy = clip.xy.astype(np.float64) / 2
    ref, area = oracle_lib.cfs_grid_general(xy, clip.off, Nx, Ny, K, L, frac_bits=F)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-L, L + 1), indexing="ij")
    keep = (np.abs(kk) <= 60) & (np.abs(ll) <= 40) & (kk ** 2 + ll ** 2 <= 45.0 ** 2)
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    Fg, a = P.forward_general(x, y, s, Nx, Ny, K, L, frac_bits=F, precision=prec,
                              band=(60, 40), radius=45.0)
    torch.cuda.synchronize()
    Fg = Fg.cpu().numpy().astype(np.complex128)
    assert int(a.item()) == area
    assert np.all(Fg[~keep] == 0)
    e = float(np.max(np.abs(Fg[keep] - ref[keep])) / abs(ref[K, L]))
    _say(f"general band {prec}: err/|F00| = {e:.3e}")
    assert e <= TOL[prec]
    with pytest.raises(P.FcfsError):
        P.forward_general(x, y, s, Nx, Ny, K, L, frac_bits=F, band=(-1, 3))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_general_autograd_low_pass(P, oracle_lib, prec):
    # loss sum |H F - G|^2 behind a pupil on a general tile through the
    # low-pass forward and its adjoint; gradient against the oracle's
    # analytic gradient with the cotangent 2 H (H F - G)
    Nx, Ny, F, K = 700, 520, 1, 30
    r = 0.35 * K
    rb = int(np.floor(r))
    clip = synth.clip(57, 1040, K, n_polygons=20)
    geom = P.Geometry(clip.xy.astype(np.float64) / 2, clip.off, Nx, K, Ny=Ny, frac_bits=F)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    H = (kk ** 2 + ll ** 2 <= r * r).astype(np.float64)
    rng = np.random.default_rng(11)
    G = H * (rng.normal(size=H.shape) + 1j * rng.normal(size=H.shape))
    Gd = torch.as_tensor(G.astype(np.complex64)).cuda()
    off = torch.zeros(geom.n_edges, dtype=torch.float32, device="cuda", requires_grad=True)
    Fv = P.FCFSFunction.apply(off, geom, prec, (rb, rb), r)
    loss = P.PupilLoss.apply(Fv, Gd, r)
    loss.backward()
    torch.cuda.synchronize()
    xy = clip.xy.astype(np.float64) / 2
    Fo, _ = oracle_lib.cfs_grid_general(xy, clip.off, Nx, Ny, K, K, frac_bits=F)
    Fh = Fv.detach().cpu().numpy().astype(np.complex128)
    assert np.all(Fh[H == 0] == 0)
    assert float(np.max(np.abs(Fh - H * Fo)) / abs(Fo[K, K])) <= TOL[prec]
    cot = 2 * H * (H * Fo - G.astype(np.complex64).astype(np.complex128))
    want = oracle_lib.edge_grad_general(xy, clip.off, Nx, Ny, K, K, cot, frac_bits=F)
    got = off.grad.cpu().numpy().astype(np.float64)
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    _say(f"general autograd low-pass {prec}: err/max|g| = {e:.3e}")
    assert e <= GTOL[prec]


@pytest.mark.parametrize("Nx,Ny,F,K,L,npol,seed", [
    (3000, 2000, 0, 300, 200, 400, 61),   # several 128 x 128 tiles, ragged in both
    (8192, 8000, 0, 64, 64, 300, 62),     # both tables at their largest
    (1000, 1000, 1, 100, 100, 300, 63),   # one shared table
])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_general_pipelined_and_eight_wave_kernels(P, oracle_lib, Nx, Ny, F, K, L, npol, seed,
                                                  prec):
    # the split precisions run the pipelined kernel; a tile variant forced on
    # the handle selects the eight-wave kernel: both against the oracle
    Mx, My = Nx << F, Ny << F
    clip = synth.clip(seed, min(Mx, My), K, L, n_polygons=npol)
    xy = clip.xy.astype(np.float64) / 2 ** F
    rng = np.random.default_rng(seed)
    lo = np.array([(k, l) for k in range(-8, 9) for l in range(-8, 9)])
    kk = np.concatenate([lo[:, 0], rng.integers(-K, K + 1, 300)])
    ll = np.concatenate([lo[:, 1], rng.integers(-L, L + 1, 300)])
    ref = oracle_lib.cfs_points_general(xy, clip.off, Nx, Ny, kk, ll, frac_bits=F)
    f00 = abs(oracle_lib.cfs_points_general(xy, clip.off, Nx, Ny, [0], [0], frac_bits=F)[0])
    h = P.default_handle()
    out = {}
    for forced in (False, True):
        if forced:
            h.set_tile(0)
        try:
            out[forced] = _gpu(P, clip.xy, clip.off, Nx, Ny, K, L, F, prec)
        finally:
            h.set_tile(-1)
        Fg, _ = out[forced]
        e = float(np.max(np.abs(Fg[kk + K, ll + L] - ref)) / f00)
        _say(f"general {Nx}x{Ny} {prec} {'eight-wave' if forced else 'pipelined'}: "
             f"err/|F00| = {e:.3e}")
        assert e <= TOL[prec]
    assert out[False][1] == out[True][1]


def test_general_low_fill_clip_near_axes(P, oracle_lib):
    # polygons in disjoint cells on a 4000 x 3000 tile with half-unit corners:
    # every coefficient with |k l| <= 160 (where the guard region widens on
    # low-fill clips) meets the split bound
    Nx, Ny, F, K = 4000, 3000, 1, 255
    clip = synth.clip(22, 8000, K, n_polygons=2000, disjoint=True)
    xy = clip.xy.astype(np.float64) / 2
    pts = [(k, l) for k in range(-K, K + 1) for l in range(-K, K + 1)
           if k and l and abs(k * l) <= 160]
    kk, ll = np.array(pts).T
    ref = oracle_lib.cfs_points_general(xy, clip.off, Nx, Ny, kk, ll, frac_bits=F)
    f00 = abs(oracle_lib.cfs_points_general(xy, clip.off, Nx, Ny, [0], [0], frac_bits=F)[0])
    for prec in ("bf16", "fp16"):
        Fg, _ = _gpu(P, clip.xy, clip.off, Nx, Ny, K, K, F, prec)
        e = np.abs(Fg[kk + K, ll + K] - ref) / f00
        w = int(np.argmax(e))
        _say(f"general low-fill clip {prec}: max err/|F00| = {e[w]:.3e} at ({kk[w]},{ll[w]})")
        assert e[w] <= TOL[prec]


def _fine_grid_clip(seed, Nx, Ny, F, K, L, npol):
    # polygons drawn on the lattice of the tile, then every loop shifted by its
    # own random sub-lattice step (a multiple of 2^-F): corners on the fine
    # grid at the fill of a lattice clip, whatever F
    clip = synth.clip(seed, max(Nx, Ny), K, L, n_polygons=npol)
    rng = np.random.default_rng(seed)
    X = clip.xy.astype(np.int64) << F
    for i in range(clip.off.size - 1):
        X[clip.off[i]:clip.off[i + 1]] += rng.integers(0, 1 << F, 2)
    return X.astype(np.int32), clip.off


@pytest.mark.parametrize("Nx,Ny,F,K,L,npol,seed", [
    (3000, 2000, 3, 40, 33, 150, 41),      # periods 24000 x 16000 (two-level tables)
    (5000, 5000, 2, 45, 45, 150, 42),      # equal periods past 8192 (one shared table)
    (2000, 9000, 0, 37, 41, 200, 43),      # one period below 8192, one above
    (1000, 700, 13, 30, 28, 60, 44),       # grid step 2^-13: periods 8192000 x 5734400
])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_general_two_level_full_grid(P, oracle_lib, Nx, Ny, F, K, L, npol, seed, prec):
    # periods past 8192 grid units: two-level twiddles, exact FP64 phases,
    # direct axis sums; every coefficient against the FP64 oracle
    Mx, My = Nx << F, Ny << F
    X, off = _fine_grid_clip(seed, Nx, Ny, F, K, L, npol)
    xy = X.astype(np.float64) / 2 ** F
    _say(f"two-level {Nx}x{Ny} F={F} (periods {Mx} x {My}) K={K} L={L} {prec}")
    ref, area = oracle_lib.cfs_grid_general(xy, off, Nx, Ny, K, L, frac_bits=F)
    Fg, a = _gpu(P, X, off, Nx, Ny, K, L, F, prec)
    assert a == area
    e = float(np.max(np.abs(Fg - ref)) / abs(ref[K, L]))
    _say(f"  err/|F00| = {e:.3e}")
    assert e <= TOL[prec]


def test_general_two_level_layout_clip(P, oracle_lib):
    # 2,000 polygons on a 4000 x 3000 tile with corners on the 1/16 grid
    # (periods 64000 x 48000), |k|, |l| <= 255: sampled coefficients, every
    # coefficient with |k l| <= 160, and the low-pass form
    Nx, Ny, F, K = 4000, 3000, 4, 255
    clip = synth.clip(45, 64000, K, n_polygons=2000)
    xy = clip.xy.astype(np.float64) / 2 ** F
    rng = np.random.default_rng(9)
    pts = [(k, l) for k in range(-K, K + 1) for l in range(-K, K + 1)
           if k and l and abs(k * l) <= 160]
    kk = np.concatenate([np.array(pts)[:, 0], rng.integers(-K, K + 1, 300), [0] * 5, [1, 2, 3]])
    ll = np.concatenate([np.array(pts)[:, 1], rng.integers(-K, K + 1, 300), [1, 2, 3, 4, 5],
                         [0] * 3])
    ref = oracle_lib.cfs_points_general(xy, clip.off, Nx, Ny, kk, ll, frac_bits=F)
    f00 = abs(oracle_lib.cfs_points_general(xy, clip.off, Nx, Ny, [0], [0], frac_bits=F)[0])
    for prec in ("fp32", "bf16"):
        Fg, _ = _gpu(P, clip.xy, clip.off, Nx, Ny, K, K, F, prec)
        e = np.abs(Fg[kk + K, ll + K] - ref) / f00
        w = int(np.argmax(e))
        _say(f"two-level layout clip {prec}: max err/|F00| = {e[w]:.3e} at ({kk[w]},{ll[w]})")
        assert e[w] <= TOL[prec]
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    Fb, _ = P.forward_general(x, y, s, Nx, Ny, K, K, frac_bits=F, precision="bf16",
                              band=(60, 60), radius=50.0)
    torch.cuda.synchronize()
    Fb = Fb.cpu().numpy().astype(np.complex128)
    ins = (np.abs(kk) <= 60) & (np.abs(ll) <= 60) & (kk ** 2 + ll ** 2 <= 2500)
    assert np.all(np.abs(Fb[kk[~ins] + K, ll[~ins] + K]) == 0)
    e = float(np.max(np.abs(Fb[kk[ins] + K, ll[ins] + K] - ref[ins])) / f00)
    _say(f"two-level layout clip low-pass bf16: err/|F00| = {e:.3e}")
    assert e <= TOL["bf16"]


@pytest.mark.parametrize("Nx,Ny,F,K,L,seed", [
    (3000, 2000, 3, 37, 45, 61),      # periods 24000 x 16000
    (5000, 5000, 2, 40, 40, 62),      # equal periods past 8192 (one table)
    (1000, 700, 13, 30, 28, 63),      # periods 8192000 x 5734400 (grid step 2^-13)
])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_general_two_level_adjoint(P, oracle_lib, Nx, Ny, F, K, L, seed, prec):
    X, off = _fine_grid_clip(seed, Nx, Ny, F, K, L, 40)
    xy = X.astype(np.float64) / 2 ** F
    G = _rand_G(K, L, seed)
    want = oracle_lib.edge_grad_general(xy, off, Nx, Ny, K, L, G.astype(np.complex64),
                                        frac_bits=F)
    x, y, s, he, ve = P.loops_to_corners(X, off)
    Gd = torch.as_tensor(G.astype(np.complex64)).cuda()
    _say(f"two-level adjoint {Nx}x{Ny} F={F} K={K} L={L} {prec}")
    gx, gy = P.adjoint_general(x, y, s, Nx, Ny, K, L, Gd, frac_bits=F, precision=prec)
    got = P.edge_grad(gx, gy, he, ve, x.size).cpu().numpy().astype(np.float64)
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    _say(f"  err/max|g| = {e:.3e}")
    assert e <= GTOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_general_two_level_autograd(P, oracle_lib, prec):
    # edges moved by multiples of 2^-10 on a 600 x 420 tile (periods 614400 x
    # 430080): loss sum |F|^2, forward and gradient against the oracle at the
    # moved corners
    Nx, Ny, F, K = 600, 420, 10, 24
    clip = synth.clip(57, 420, K, n_polygons=12)
    geom = P.Geometry(clip.xy, clip.off, Nx, K, Ny=Ny, frac_bits=F)
    rng = np.random.default_rng(10)
    offs = rng.integers(-700, 701, geom.n_edges) / 1024.0
    off = torch.tensor(offs, dtype=torch.float32, device="cuda", requires_grad=True)
    Fv = P.FCFSFunction.apply(off, geom, prec)
    (Fv.abs() ** 2).sum().backward()
    torch.cuda.synchronize()
    xy = clip.xy.astype(np.float64).copy()
    for m in range(clip.off.size - 1):
        a0, a1 = clip.off[m], clip.off[m + 1]
        for e in range(a0, a1):
            b = a0 + (e - a0 + 1) % (a1 - a0)
            axis = 0 if clip.xy[e, 0] == clip.xy[b, 0] else 1
            xy[e, axis] += offs[e]
            xy[b, axis] += offs[e]
    ref, _ = oracle_lib.cfs_grid_general(xy, clip.off, Nx, Ny, K, K, frac_bits=F)
    Fg = Fv.detach().cpu().numpy().astype(np.complex128)
    ef = float(np.max(np.abs(Fg - ref)) / abs(ref[K, K]))
    want = oracle_lib.edge_grad_general(xy, clip.off, Nx, Ny, K, K, 2 * ref, frac_bits=F)
    got = off.grad.cpu().numpy().astype(np.float64)
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    _say(f"two-level autograd {prec}: F err/|F00| = {ef:.3e}, grad err/max|g| = {e:.3e}")
    assert ef <= TOL[prec]
    assert e <= GTOL[prec]


def test_general_two_level_adjoint_limit(P):
    # the adjoint takes periods up to 2^23; 3000 x 2^12 is past that
    clip = synth.clip(46, 3000, 20, n_polygons=20)
    x, y, s, _, _ = P.loops_to_corners(clip.xy.astype(np.int64) << 12, clip.off)
    g = torch.zeros((41, 41), dtype=torch.complex64, device="cuda")
    with pytest.raises(P.FcfsError) as ei:
        P.adjoint_general(x, y, s, 3000, 3000, 20, 20, g, frac_bits=12)
    assert ei.value.status == -4


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_general_batch_graph(P, oracle_lib, prec):
    # clips of different periods, grid steps and cut-offs (two of them past
    # 8192 grid units) in one plan: the oracle agrees with the first pass, the
    # single calls agree with it to the precision's bound (the batch chooses
    # its own split counts, so the FP32 sums are taken in another order), and
    # replays repeat it bit for bit
    specs = [(3000, 2000, 0, 40, 33, 150, 71), (750, 1000, 2, 37, 45, 150, 72),
             (1000, 700, 13, 30, 28, 60, 73), (3000, 2000, 3, 41, 29, 100, 74),
             (7, 5, 3, 30, 29, 6, 75)]
    clips, refs = [], []
    for Nx, Ny, F, K, L, npol, seed in specs:
        if Nx < 100:  # a tiny tile: polygons drawn on the grid itself
            c = synth.clip(seed, max(Nx, Ny) << F, K, L, n_polygons=npol)
            X, off = c.xy, c.off
        else:
            X, off = _fine_grid_clip(seed, Nx, Ny, F, K, L, npol)
        x, y, s, _, _ = P.loops_to_corners(X, off)
        clips.append((x, y, s, Nx, Ny, K, L, F))
        refs.append(oracle_lib.cfs_grid_general(X.astype(np.float64) / 2 ** F, off, Nx, Ny, K, L,
                                                frac_bits=F))
    _say(f"general batch of {len(clips)} clips (graph), {prec}")
    b = P.GeneralBatch(clips, precision=prec)
    torch.cuda.synchronize()
    eager = [f.cpu().numpy().copy() for f in b.F]
    for i, (x, y, s, Nx, Ny, K, L, F) in enumerate(clips):
        Fs, a = P.forward_general(x, y, s, Nx, Ny, K, L, frac_bits=F, precision=prec)
        torch.cuda.synchronize()
        ref, area = refs[i]
        d = float(np.max(np.abs(Fs.cpu().numpy().astype(np.complex128) - eager[i]))
                  / abs(ref[K, L]))
        assert d <= TOL[prec], (i, d)
        assert int(b.area[i].item()) == area
        e = float(np.max(np.abs(eager[i].astype(np.complex128) - ref)) / abs(ref[K, L]))
        assert e <= TOL[prec], (i, e)
    for _ in range(2):
        for f in b.F:
            f.zero_()
        b.run()
        torch.cuda.synchronize()
        for i in range(len(clips)):
            assert np.array_equal(b.F[i].cpu().numpy(), eager[i]), i
    b.close()


def test_general_batch_many_periods_and_rewritten_corners(P, oracle_lib):
    # 20 clips with 40 distinct periods, more than the handle keeps in its
    # table cache (the plan pins its own); a single call on yet another period
    # afterwards has to build its table beside the pinned ones.  Then the
    # corners of every clip are shifted in place (same corner count) and the
    # replay, which reads the current corner contents, is checked against
    # single calls on the shifted corners and, for three clips, the oracle.
    specs = []
    for i in range(20):
        Nx, Ny = 200 + 37 * i, 310 + 23 * i
        specs.append((Nx, Ny, i % 3, 20, 18, 12, 600 + i))
    clips, data = [], []
    for Nx, Ny, F, K, L, npol, seed in specs:
        X, off = _fine_grid_clip(seed, Nx, Ny, F, K, L, npol)
        x, y, s, _, _ = P.loops_to_corners(X, off)
        clips.append((x, y, s, Nx, Ny, K, L, F))
        data.append((X, off))
    _say(f"general batch of {len(clips)} clips, {2 * len(clips)} distinct periods")
    b = P.GeneralBatch(clips, precision="bf16")
    torch.cuda.synchronize()
    Fo, _ = _gpu(P, *_fine_grid_clip(700, 333, 444, 1, 20, 18, 12), 333, 444, 20, 18, 1, "bf16")
    assert np.isfinite(Fo).all()
    for i, (Nx, Ny, F, K, L, npol, seed) in enumerate(specs):
        X, off = data[i]
        ref, area = oracle_lib.cfs_grid_general(X.astype(np.float64) / 2 ** F, off, Nx, Ny, K, L,
                                                frac_bits=F)
        e = float(np.max(np.abs(b.F[i].cpu().numpy().astype(np.complex128) - ref)) / abs(ref[K, L]))
        assert e <= TOL["bf16"], (i, e)
        assert int(b.area[i].item()) == area
    # shift every clip by its own grid step (corners keep their count)
    for i, (x, y, s) in enumerate(b.corners):
        x.add_(3 + i)
        y.sub_(5 + 2 * i)
    b.run()
    torch.cuda.synchronize()
    for i, (x, y, s) in enumerate(b.corners):
        Nx, Ny, F, K, L, npol, seed = specs[i]
        Fs, a = P.forward_general(x, y, s, Nx, Ny, K, L, frac_bits=F, precision="bf16")
        torch.cuda.synchronize()
        Fs = Fs.cpu().numpy().astype(np.complex128)
        d = float(np.max(np.abs(Fs - b.F[i].cpu().numpy())) / abs(Fs[K, L]))
        assert d <= TOL["bf16"], (i, d)
        assert int(b.area[i].item()) == int(a.item())
        if i in (0, 7, 19):
            X, off = data[i]
            Xs = X.astype(np.float64) + np.array([3 + i, -(5 + 2 * i)], dtype=np.float64)
            ref, area = oracle_lib.cfs_grid_general(Xs / 2 ** F, off, Nx, Ny, K, L, frac_bits=F)
            e = float(np.max(np.abs(b.F[i].cpu().numpy().astype(np.complex128) - ref))
                      / abs(ref[K, L]))
            assert e <= TOL["bf16"], (i, e)
            assert int(b.area[i].item()) == area
    b.close()


@pytest.mark.parametrize("K,L", [(600, 300), (200, 130)])
def test_general_two_level_axes_wide_bands(P, oracle_lib, K, L):
    # periods past 8192 grid units with bands of 512-frequency (K = 600: two
    # blocks, the second starting at f0 = 512) and 256-frequency axis blocks:
    # every axis coefficient F[k, 0], F[0, l] and a sample of the rest against
    # the oracle
    Nx, Ny, F = 1500, 1100, 5
    X, off = _fine_grid_clip(47, Nx, Ny, F, K, L, 40)
    xy = X.astype(np.float64) / 2 ** F
    rng = np.random.default_rng(11)
    kk = np.concatenate([np.arange(1, K + 1), -np.arange(1, K + 1), np.zeros(L, int),
                         np.zeros(L, int), rng.integers(-K, K + 1, 400)])
    ll = np.concatenate([np.zeros(K, int), np.zeros(K, int), np.arange(1, L + 1),
                         -np.arange(1, L + 1), rng.integers(-L, L + 1, 400)])
    ref = oracle_lib.cfs_points_general(xy, off, Nx, Ny, kk, ll, frac_bits=F)
    f00 = abs(oracle_lib.cfs_points_general(xy, off, Nx, Ny, [0], [0], frac_bits=F)[0])
    _say(f"two-level axes {Nx}x{Ny} F={F} K={K} L={L}: {off.size - 1} polygons")
    for prec in ("fp32", "bf16"):
        Fg, _ = _gpu(P, X, off, Nx, Ny, K, L, F, prec)
        e = np.abs(Fg[kk + K, ll + L] - ref) / f00
        w = int(np.argmax(e))
        _say(f"  {prec}: max err/|F00| = {e[w]:.3e} at ({kk[w]},{ll[w]})")
        assert e[w] <= TOL[prec]
