"""The entry point that allocates nothing (fcfs_forward_noalloc) against the
workspace entry point (fcfs_forward): same kernels, so the same bits, on two
calls in a row, the second with a smaller clip; a clip past the library's
scratch is refused.  Called through the C ABI on cuda:0."""
import ctypes

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


def _call(P, h, clip, prec, noalloc):
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    x, y, s = (torch.as_tensor(a).cuda() for a in (x, y, s))
    F = torch.full((2 * clip.K + 1, 2 * clip.L + 1), complex(7.0, 7.0), dtype=torch.complex64,
                   device="cuda")
    a = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    c = P._clip(x, y, s, x.numel(), clip.T, clip.K, clip.L, F, a)
    if noalloc:
        st = h.lib.fcfs_forward_noalloc(h.ptr, ctypes.byref(c), P.PRECISIONS[prec])
    else:
        nb = P.workspace_size(x.numel(), clip.T, clip.K, clip.L, prec)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        st = h.lib.fcfs_forward(h.ptr, ctypes.byref(c), P.PRECISIONS[prec],
                                ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(nb))
    assert st == 0, h.lib.fcfs_last_error(h.ptr)
    torch.cuda.synchronize()
    return F.cpu().numpy(), int(a.item())


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_noalloc_matches_workspace_entry(P, prec):
    h = P.Handle()
    big = synth.clip(91, 8192, 511, min_vertices=200_000)   # the precision clip's size
    small = synth.clip(92, 2048, 100, n_polygons=300)       # a smaller one next
    for clip in (big, small):
        Fn, an = _call(P, h, clip, prec, True)
        Fw, aw = _call(P, h, clip, prec, False)
        print(f"noalloc {prec}: V={clip.n_vertices} T={clip.T} K={clip.K}: "
              f"max |diff| = {np.max(np.abs(Fn - Fw)):.3e}", flush=True)
        assert an == aw
        assert np.array_equal(Fn, Fw)
    h.close()


def test_noalloc_refuses_past_its_scratch(P):
    # a clip whose workspace exceeds the library's scratch: FCFS_ERR_WORKSPACE
    # before anything is enqueued
    h = P.Handle()
    V = 2_000_000
    need = P.workspace_size(V, 8192, 1023, 1023, "bf16")
    assert need > 96 << 20
    x = torch.zeros(V, dtype=torch.int32, device="cuda")
    s = torch.ones(V, dtype=torch.int8, device="cuda")
    F = torch.empty((2047, 2047), dtype=torch.complex64, device="cuda")
    a = torch.empty(1, dtype=torch.int64, device="cuda")
    c = P._clip(x, x, s, V, 8192, 1023, 1023, F, a)
    st = h.lib.fcfs_forward_noalloc(h.ptr, ctypes.byref(c), P.PRECISIONS["bf16"])
    assert st == -5
    assert b"scratch" in h.lib.fcfs_last_error(h.ptr)
    # the handle still works
    clip = synth.clip(93, 1024, 40, n_polygons=40)
    Fn, _ = _call(P, h, clip, "bf16", True)
    Fw, _ = _call(P, h, clip, "bf16", False)
    assert np.array_equal(Fn, Fw)
    h.close()
