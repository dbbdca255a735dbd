"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, canonicalises loops into signed corners, validates its arguments and
sizes workspaces.  No device work is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from tests import helpers as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1010_5562_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libfcfs.so is not built (run __graft_entry__.build())")
    return _lib.load()


def _declared():
    # every function the headers under include/ declare
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(fcfs_\w+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol(lib):
    from paper_1010_5562_amd import _lib

    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_status_strings(lib):
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.fcfs_status_string(st)
    assert lib.fcfs_last_error(None) is not None


def test_loops_to_corners_signs_match_raster_corners():
    import paper_1010_5562_amd as P

    c = synth.clip(21, 256, 10, n_polygons=1)
    x, y, s, he, ve = P.loops_to_corners(c.xy, c.off)
    assert np.array_equal(x, c.xy[:, 0]) and np.array_equal(y, c.xy[:, 1])
    # corner weights of the rasterised polygon (independent of the edge walk)
    W = H.corner_image(H.raster(c.xy, c.off, 256))
    assert np.array_equal(W[x, y], s.astype(np.int64))
    assert int(np.count_nonzero(W)) == c.n_vertices
    # edge maps: hedge[v] is the horizontal edge at v, vedge[v] the vertical one
    n = c.n_vertices
    for v in range(n):
        for e, horiz in ((he[v], True), (ve[v], False)):
            a, b = c.xy[e], c.xy[(e + 1) % n]
            assert v in (e, (e + 1) % n)
            assert (a[1] == b[1]) == horiz


def test_loops_to_corners_counter_clockwise_and_multi():
    import paper_1010_5562_amd as P

    r1 = synth.rectangle_loop(0, 0, 5, 3)
    r2 = synth.rectangle_loop(10, 10, 12, 20)[::-1]  # counter-clockwise
    xy = np.concatenate([r1, r2])
    x, y, s, he, ve = P.loops_to_corners(xy, [0, 4, 8])
    # sum s x y is the total area for both orientations
    assert int(np.sum(s.astype(np.int64) * x * y)) == 15 + 20
    # per polygon the signs sum to zero
    assert s[:4].sum() == 0 and s[4:].sum() == 0


@pytest.mark.parametrize(
    "xy,off,status",
    [
        ([[0, 0], [0, 5], [5, 5]], [0, 3], -2),
        ([[0, 0], [0, 5], [5, 6], [5, 0]], [0, 4], -2),
        ([[0, 0], [0, 5], [0, 9], [5, 9], [5, 0], [3, 0]], [0, 6], -2),
        ([[0, 0], [0, 0], [5, 0], [5, 0]], [0, 4], -2),
        ([[0, 0], [0, 1 << 30], [5, 1 << 30], [5, 0]], [0, 4], -3),
    ],
)
def test_loops_to_corners_rejects(xy, off, status):
    import paper_1010_5562_amd as P

    with pytest.raises(P.FcfsError) as ei:
        P.loops_to_corners(np.array(xy), off)
    assert ei.value.status == status


def test_workspace_sizes():
    import paper_1010_5562_amd as P

    a = P.workspace_size(40000, 4096, 255, 255, "fp32")
    b = P.workspace_size(200000, 8192, 511, 511, "bf16")
    assert 0 < a < b < 1 << 31
    assert P.workspace_size(0, 2, 0, 0, "fp16") > 0
    for t in range(len(P.tile_variants())):
        assert P.workspace_size(1000, 1024, 63, 63, "bf16", tile=t) > 0
    with pytest.raises(P.FcfsError) as ei:
        P.workspace_size(10, 1000, 4, 4)  # not a power of two
    assert ei.value.status == -4
    with pytest.raises(P.FcfsError) as ei:
        P.workspace_size(10, 16384, 4, 4)
    assert ei.value.status == -4
    with pytest.raises(P.FcfsError) as ei:
        P.workspace_size(10, 1024, 5000, 4)
    assert ei.value.status == -4
    with pytest.raises(P.FcfsError) as ei:
        P.workspace_size(10, 1024, -1, 4)
    assert ei.value.status == -1


def test_general_workspace_sizes(lib):
    # the low-pass form needs less than the full grid; invalid bands, radii
    # and periods are rejected before any device work
    from paper_1010_5562_amd import _lib

    c = _lib.FcfsGClip(None, None, None, 200000, 8000, 6000, 0, 511, 511, None, None)
    full, band = ctypes.c_size_t(0), ctypes.c_size_t(0)
    for prec in (0, 1, 2):
        assert lib.fcfs_general_workspace_size(ctypes.byref(c), prec, ctypes.byref(full)) == 0
        assert lib.fcfs_general_band_workspace_size(ctypes.byref(c), 100, 100, 90.0, prec,
                                                    ctypes.byref(band)) == 0
        assert 0 < band.value < full.value < 1 << 32
    assert lib.fcfs_general_band_workspace_size(ctypes.byref(c), -1, 3, -1.0, 1,
                                                ctypes.byref(band)) == -1
    assert lib.fcfs_general_band_workspace_size(ctypes.byref(c), 3, 3, float("nan"), 1,
                                                ctypes.byref(band)) == -1
    # periods past 8192 take the two-level tables (the adjoint up to 2^23);
    # past 2^24 they are rejected
    c.Nx = 9000
    assert lib.fcfs_general_workspace_size(ctypes.byref(c), 1, ctypes.byref(full)) == 0
    assert lib.fcfs_general_adjoint_workspace_size(ctypes.byref(c), 1, ctypes.byref(full)) == 0
    c.Nx, c.Ny, c.frac_bits = 3000, 3000, 12
    assert lib.fcfs_general_workspace_size(ctypes.byref(c), 1, ctypes.byref(full)) == 0
    assert lib.fcfs_general_adjoint_workspace_size(ctypes.byref(c), 1, ctypes.byref(full)) == -4
    c.Ny, c.frac_bits = 6000, 0
    c.Nx, c.frac_bits = 4097, 12
    assert lib.fcfs_general_workspace_size(ctypes.byref(c), 1, ctypes.byref(full)) == -4
    c.Nx = 4096
    assert lib.fcfs_general_workspace_size(ctypes.byref(c), 1, ctypes.byref(full)) == -4
    c.Ny = 4096
    assert lib.fcfs_general_workspace_size(ctypes.byref(c), 1, ctypes.byref(full)) == 0


def test_general_batch_workspace_size(lib):
    # one 256-byte aligned slice per clip; an FP32 batch keeps the single-clip
    # layouts (a captured sequence of single-clip forwards), a split-precision
    # batch sizes its own split counts (one launch per step); an empty batch
    # is rejected
    from paper_1010_5562_amd import _lib

    specs = [(200000, 8000, 6000, 0, 511, 511), (3000, 3000, 2000, 3, 40, 33),
             (500, 7, 5, 3, 30, 29)]
    cs = (_lib.FcfsGClip * 3)(*[_lib.FcfsGClip(None, None, None, V, Nx, Ny, F, K, L, None, None)
                                for V, Nx, Ny, F, K, L in specs])
    each = []
    for c in cs:
        n = ctypes.c_size_t(0)
        assert lib.fcfs_general_workspace_size(ctypes.byref(c), 0, ctypes.byref(n)) == 0
        each.append((n.value + 255) // 256 * 256)
    total = ctypes.c_size_t(0)
    assert lib.fcfs_general_batch_workspace_size(cs, 3, 0, ctypes.byref(total)) == 0
    assert total.value == sum(each)
    t1, t2 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.fcfs_general_batch_workspace_size(cs, 3, 1, ctypes.byref(t1)) == 0
    assert lib.fcfs_general_batch_workspace_size(cs, 3, 1, ctypes.byref(t2)) == 0
    assert t1.value == t2.value and t1.value % 256 == 0
    # at least the corner records, magics and one 128 x 128 partial per clip
    assert t1.value >= sum(16 * V + 4 * 4 * 128 * 128 for V, *_ in specs)
    assert lib.fcfs_general_batch_workspace_size(cs, 0, 1, ctypes.byref(total)) == -1


def test_pupil_step_workspace_size(lib):
    n = ctypes.c_size_t(0)
    assert lib.fcfs_pupil_step_workspace_size(100000, 4096, 255, 255, 89, 89, 89.25, 1,
                                              ctypes.byref(n)) == 0
    full = ctypes.c_size_t(0)
    assert lib.fcfs_pupil_step_workspace_size(100000, 4096, 255, 255, 255, 255, -1.0, 1,
                                              ctypes.byref(full)) == 0
    # moved corners, spectrum, cotangent and per-corner gradients come on top
    assert full.value >= n.value > 2 * 511 * 511 * 8 + 4 * 4 * 100000
    assert lib.fcfs_pupil_step_workspace_size(100, 1000, 8, 8, 8, 8, -1.0, 1,
                                              ctypes.byref(n)) == -4  # T not a power of two
    assert lib.fcfs_pupil_step_workspace_size(100, 1024, 8, 8, -1, 8, -1.0, 1,
                                              ctypes.byref(n)) == -1
    assert lib.fcfs_pupil_step_workspace_size(100, 1024, 8, 8, 8, 8, float("nan"), 1,
                                              ctypes.byref(n)) == -1


def test_haar_workspace_size(lib):
    from paper_1010_5562_amd._lib import FcfsHaarClip

    def size(M, Nx=4096, Ny=4096, J=12):
        c = FcfsHaarClip(None, None, None, None, 10 * M, M, Nx, Ny, J, None, None, None)
        n = ctypes.c_size_t(0)
        st = lib.fcfs_haar_workspace_size(ctypes.byref(c), ctypes.byref(n))
        return st, n.value

    # control words, 64 copies of the 64 x 64 int64 coarse block, a task count
    # per polygon and the extra-task list (at least 4096 entries)
    st, n0 = size(0)
    assert st == 0 and n0 >= 256 + 64 * 64 * 64 * 8 + 8 * 4096
    st, n1 = size(100000)
    assert st == 0 and n1 >= 256 + 64 * 64 * 64 * 8 + 4 * 100000 + 8 * 100000
    # the size depends on M only
    assert size(100000, 1024, 512, 9)[1] == n1
    assert size(10, 24, 24, 4)[0] == -1      # 2^J does not divide the tile
    assert size(10, 8192, 8192, 14)[0] == -4  # J past 13


def test_null_handle_is_rejected(lib):
    from paper_1010_5562_amd import _lib

    c = _lib.FcfsClip()
    st = lib.fcfs_forward(None, ctypes.byref(c), 0, None, 0)
    assert st == -1


def test_log_and_roctx_switches(lib):
    # FCFS_LOG=1 prints one line per call to stderr; FCFS_ROCTX=1 opens the
    # roctx library when present and brackets the call with a range (a host
    # call is enough to exercise both without a GPU)
    import subprocess
    import sys

    code = ("import sys; sys.path.insert(0, %r)\n"
            "import synth, paper_1010_5562_amd as P\n"
            "c = synth.clip(1, 1024, 10, n_polygons=3)\n"
            "P.loops_to_corners(c.xy, c.off)\n") % ROOT
    env = dict(os.environ, FCFS_LOG="1", FCFS_ROCTX="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "[fcfs] fcfs_loops_to_corners 3 loops" in r.stderr
    env.pop("FCFS_LOG")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and "[fcfs]" not in r.stderr


def test_auto_form_choice():
    # FCFS_AUTO: the lattice form where its L T log2 T work is well below the
    # contraction's 24 (K+1)(L+1) V flop, the split contraction otherwise, the
    # direct form for small problems; sizes only (no device needed)
    import paper_1010_5562_amd as P

    assert P.plan_info(200_012, 8192, 511, 511, "auto")["form"] == "lattice"
    assert P.plan_info(32_122, 4096, 255, 255, "auto")["form"] == "contraction"
    assert P.plan_info(64, 2048, 64, 64, "auto")["form"] == "direct"
    assert P.plan_info(200_012, 8192, 511, 511, "bf16")["form"] == "contraction"
    # the workspace follows the form taken
    assert P.workspace_size(200_012, 8192, 511, 511, "auto") != \
        P.workspace_size(200_012, 8192, 511, 511, "bf16")
