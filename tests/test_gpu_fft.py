"""GPU parity of the lattice (FFT) form against the FP64 oracle, and full-grid
parity of the MFMA contraction against the lattice form at full size.

The lattice form computes in FP64 and rounds to complex64 at the end, so its
error bar relative to |F[0,0]| is the FP32 rounding of the output (1e-7)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FFT = 1e-7


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_5562_amd as P

    torch.cuda.set_device(0)
    return P


def _say(msg):
    print(msg, flush=True)


def _fft(P, xy, off, T, K, L):
    x, y, s, _, _ = P.loops_to_corners(xy, off)
    F, a = P.forward_fft(x, y, s, T, K, L)
    torch.cuda.synchronize()
    return F.cpu().numpy().astype(np.complex128), int(a.item())


@pytest.mark.parametrize("T,K,L,npol", [(1024, 150, 97, 211), (256, 40, 40, 30), (2, 3, 2, 5)])
def test_fft_form_full_grid(P, oracle_lib, T, K, L, npol):
    # drawn on a tile of at least 300 units, evaluated with period T (the CFS
    # of the periodisation when the polygons exceed the tile)
    clip = synth.clip(51, max(T, 300), K, L, n_polygons=npol)
    ref, area = oracle_lib.cfs_grid(clip.xy, clip.off, T, K, L)
    F, a = _fft(P, clip.xy, clip.off, T, K, L)
    assert a == area
    e = float(np.max(np.abs(F - ref)) / abs(ref[K, L]))
    _say(f"lattice form T={T} K={K} L={L}: err/|F00| = {e:.3e}")
    assert e <= TOL_FFT


def test_fft_form_wraps_and_negative_coordinates(P, oracle_lib):
    # K beyond T / 2 (the DFT is periodic in k) and coordinates outside [0, T)
    clip = synth.clip(52, 300, 100, 70, n_polygons=12)
    xy = synth.shift_loops(clip.xy, -37, 91)
    ref, area = oracle_lib.cfs_grid(xy, clip.off, 64, 100, 70)
    F, a = _fft(P, xy, clip.off, 64, 100, 70)
    assert a == area
    assert float(np.max(np.abs(F - ref)) / abs(ref[100, 70])) <= TOL_FFT


def test_fft_form_empty(P):
    e = np.zeros(0, np.int32)
    F, a = P.forward_fft(e, e, e.astype(np.int8), 512, 5, 4)
    torch.cuda.synchronize()
    assert int(a.item()) == 0 and bool((F == 0).all())


def test_contraction_full_grid_against_lattice_form(P, oracle_lib):
    # precision clip (200k corners, T = 8192, |k|,|l| <= 511): the lattice
    # form is pinned to the oracle on sampled points, then serves as the
    # full-grid reference of the split-bf16 and FP32 contractions
    T, K = 8192, 511
    clip = synth.clip(3, T, K, min_vertices=200_000)
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    Ff, _ = P.forward_fft(x, y, s, T, K, K)
    torch.cuda.synchronize()
    Ff = Ff.cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(9)
    lo = np.array([(k, l) for k in range(-8, 9) for l in range(-8, 9)])
    kk = np.concatenate([lo[:, 0], rng.integers(-K, K + 1, 300)])
    ll = np.concatenate([lo[:, 1], rng.integers(-K, K + 1, 300)])
    ref = oracle_lib.cfs_points(clip.xy, clip.off, T, kk, ll)
    f00 = abs(oracle_lib.cfs_points(clip.xy, clip.off, T, [0], [0])[0])
    e_fft = float(np.max(np.abs(Ff[kk + K, ll + K] - ref)) / f00)
    _say(f"lattice form vs oracle on {kk.size} points: {e_fft:.3e}")
    assert e_fft <= TOL_FFT
    for prec, tol in (("bf16", 1e-5), ("fp32", 1e-6)):
        F, _ = P.forward(x, y, s, T, K, K, precision=prec)
        torch.cuda.synchronize()
        e = float(np.max(np.abs(F.cpu().numpy().astype(np.complex128) - Ff)) / f00)
        _say(f"{prec} contraction vs lattice form, full 1023 x 1023 grid: {e:.3e}")
        assert e <= tol


@pytest.mark.parametrize("case", ["precision", "layout"])
def test_auto_form_takes_the_cheaper_form(P, oracle_lib, case):
    # precision "auto": the result is bit for bit the form the plan names
    # (the lattice form at the precision clip's size, the split-bf16
    # contraction at the layout clip's) and meets the split bound
    if case == "precision":
        clip = synth.clip(3, 8192, 511, min_vertices=200_000)
    else:
        clip = synth.clip(2, 4096, 255, n_polygons=2000)
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    form = P.plan_info(x.size, clip.T, clip.K, clip.L, "auto")["form"]
    Fa, aa = P.forward(x, y, s, clip.T, clip.K, clip.L, precision="auto")
    if form == "lattice":
        Fr, ar = P.forward_fft(x, y, s, clip.T, clip.K, clip.L)
    else:
        Fr, ar = P.forward(x, y, s, clip.T, clip.K, clip.L, precision="bf16")
    torch.cuda.synchronize()
    print(f"auto at V={x.size} T={clip.T} K={clip.K}: {form}", flush=True)
    assert torch.equal(Fa, Fr) and int(aa.item()) == int(ar.item())
    kk = np.array([0, 1, 3, -7, 200, -511 if clip.K >= 511 else -255])
    ll = np.array([0, 2, -5, 9, -100, 17])
    ref = oracle_lib.cfs_points(clip.xy, clip.off, clip.T, kk, ll)
    e = float(np.max(np.abs(Fa.cpu().numpy()[kk + clip.K, ll + clip.L] - ref)) / abs(ref[0]))
    assert e <= 1e-5
