"""GPU parity of the pruned continuous Haar transform (fcfs_haar) against the
PCHT oracle.

The integer pyramid U must match the oracle bit for bit (areas are exact
integers on both sides), and so must the number of cells visited.  W is
U * 2^j / sqrt(Nx Ny): exact on both sides for square power-of-two tiles,
otherwise one rounding apart at most."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_5562_amd as P

    torch.cuda.set_device(0)
    return P


def _say(msg):
    print(msg, flush=True)


def _gpu(P, xy, off, Nx, Ny, J):
    x, y, s, _, _ = P.loops_to_corners(xy, off)
    U, W, st = P.haar(x, y, s, off, Nx, Ny, J, stats=True)
    torch.cuda.synchronize()
    return U.cpu().numpy(), W.cpu().numpy(), st.cpu().numpy()


def _check(P, oracle_lib, xy, off, Nx, Ny, J, what, exact_w=True):
    _say(f"haar {what}: {off.size - 1} polygons, {int(off[-1])} corners, {Nx}x{Ny}, J={J}")
    Uo, Wo, nodes = oracle_lib.pcht(xy, off, Nx, Ny, J)
    U, W, st = _gpu(P, xy, off, Nx, Ny, J)
    assert np.array_equal(U, Uo), f"{what}: {np.count_nonzero(U != Uo)} integer sums differ"
    assert int(st[0]) == nodes
    if exact_w:
        assert np.array_equal(W, Wo)
    else:
        assert np.max(np.abs(W - Wo)) <= 2 * np.finfo(float).eps * np.max(np.abs(Wo))
    return U, st


def _staircase(n_steps, step=3, x0=5, y0=7):
    """One clockwise staircase loop with 2 n_steps + 2 corners."""
    pts = [(x0, y0)]
    for i in range(n_steps):
        pts.append((x0 + i * step, y0 + (i + 1) * step))
        pts.append((x0 + (i + 1) * step, y0 + (i + 1) * step))
    pts.append((x0 + n_steps * step, y0))
    xy = np.array(pts, dtype=np.int32)
    return xy, np.array([0, xy.shape[0]], dtype=np.int64)


def test_haar_layout_clip_full_pyramid(P, oracle_lib):
    # 2,000 polygons on a 4096 tile, the full 12-level pyramid
    clip = synth.clip(2, 4096, 0, n_polygons=2000)
    U, st = _check(P, oracle_lib, clip.xy, clip.off, 4096, 4096, 12, "layout clip")
    _say(f"  cells visited {int(st[0])}, nonzero coefficients {np.count_nonzero(U)}")


@pytest.mark.parametrize("Nx,Ny,J,seed", [(2048, 1024, 10, 7), (768, 640, 7, 8), (512, 512, 4, 9)])
def test_haar_rectangular_and_shallow_tiles(P, oracle_lib, Nx, Ny, J, seed):
    clip = synth.clip(seed, max(Nx, Ny), 0, n_polygons=300)
    exact = Nx == Ny and (Nx & (Nx - 1)) == 0
    _check(P, oracle_lib, clip.xy, clip.off, Nx, Ny, J, f"seed {seed}", exact_w=exact)


def test_haar_polygons_across_the_tile_edge_and_reversed(P, oracle_lib):
    clip = synth.clip(10, 1024, 0, n_polygons=200)
    xy = synth.shift_loops(clip.xy, -300, 250)
    _check(P, oracle_lib, xy, clip.off, 1024, 1024, 10, "shifted")
    rev = np.concatenate([xy[clip.off[m]:clip.off[m + 1]][::-1]
                          for m in range(clip.off.size - 1)])
    _check(P, oracle_lib, rev, clip.off, 1024, 1024, 10, "shifted, counter-clockwise")


def test_haar_polygon_larger_than_one_staging_pass(P, oracle_lib):
    # 3,002 corners: the corner list is staged in several passes per cell batch
    xy, off = _staircase(1500, step=2)
    _check(P, oracle_lib, xy, off, 4096, 4096, 12, "staircase")
    # together with small polygons in the same launch
    c = synth.clip(11, 4096, 0, n_polygons=50)
    xy2 = np.concatenate([xy, c.xy + 0])
    off2 = np.concatenate([off, off[-1] + c.off[1:]])
    _check(P, oracle_lib, xy2, off2, 8192, 8192, 13, "staircase + clip, J=13")


def test_haar_degenerate_sizes(P, oracle_lib):
    sq = synth.rectangle_loop(1, 2, 5, 9)
    off = np.array([0, 4], dtype=np.int64)
    for Nx, Ny, J in ((16, 16, 0), (1, 1, 0), (8, 16, 3), (2, 2, 1)):
        _check(P, oracle_lib, sq, off, Nx, Ny, J, f"rectangle {Nx}x{Ny} J={J}",
               exact_w=(Nx == Ny))
    # no polygons at all
    e = np.zeros(0, np.int32)
    U, W, st = P.haar(e, e, e.astype(np.int8), np.zeros(1, np.int64), 64, 64, 6, stats=True)
    torch.cuda.synchronize()
    assert not U.any() and not W.any() and int(st[0]) == 0


@pytest.mark.parametrize("J", [10, 5])
def test_haar_overlapping_polygons_integer_only_and_repeated(P, oracle_lib, J):
    # 3,000 overlapping rectangles, some across the tile edge: every wave takes
    # several polygons and the coarse levels collect thousands of contributions
    # (summed in per-workgroup copies, then added into U).  Calls without W
    # (coarse block added by its own launch) and repeated calls on the same
    # workspace, over a U that holds stale values, give the oracle's sums.
    rng = np.random.default_rng(12)
    n, T = 3000, 1024
    x1, y1 = rng.integers(-40, T, n), rng.integers(-40, T, n)
    w, h = rng.integers(1, 200, n), rng.integers(1, 200, n)
    loops = [synth.rectangle_loop(int(a), int(b), int(a + c), int(b + d))
             for a, b, c, d in zip(x1, y1, w, h)]
    xy = np.concatenate(loops).astype(np.int32)
    off = np.concatenate([[0], np.cumsum([lp.shape[0] for lp in loops])]).astype(np.int64)
    _say(f"haar overlapping rectangles: {n} polygons, {T}x{T}, J={J}")
    Uo, Wo, nodes = oracle_lib.pcht(xy, off, T, T, J)
    x, y, s, _, _ = P.loops_to_corners(xy, off)
    U = torch.full((1 << J, 1 << J), 12345, dtype=torch.int64, device="cuda")
    for rep in range(2):
        U2, W2, st = P.haar(x, y, s, off, T, T, J, out_U=U, coefficients=False, stats=True)
        torch.cuda.synchronize()
        assert W2 is None
        assert np.array_equal(U.cpu().numpy(), Uo), f"U only, call {rep}"
        assert int(st[0].item()) == nodes
    U3, W3, _ = P.haar(x, y, s, off, T, T, J, out_U=U)
    torch.cuda.synchronize()
    assert np.array_equal(U3.cpu().numpy(), Uo)
    assert np.array_equal(W3.cpu().numpy(), Wo)


def test_haar_rejects_bad_sizes(P):
    sq = synth.rectangle_loop(0, 0, 3, 3)
    x, y, s, _, _ = P.loops_to_corners(sq, np.array([0, 4]))
    off = np.array([0, 4])
    for Nx, Ny, J in ((24, 24, 4), (16384, 16384, 2), (8192, 8192, 14), (0, 8, 0)):
        with pytest.raises(P.FcfsError):
            P.haar(x, y, s, off, Nx, Ny, J)
