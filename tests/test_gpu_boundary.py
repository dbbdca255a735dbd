"""Error paths and lifetimes at the C ABI: workspaces that are too small or
misaligned, a stream the caller is capturing, a change of stream between
calls on one handle, plans that outlive their
handle, general-tile batches past the handle's table cache, and replays that
recompute from rewritten corners.  Every case calls the library through the
C ABI (ctypes) on cuda:0; the error cases enqueue nothing on the device."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-5


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_5562_amd as P

    torch.cuda.set_device(0)
    return P


def _say(msg):
    print(msg, flush=True)


def _forward_call(P, h, clip, prec, ws, nbytes):
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    x, y, s = (torch.as_tensor(a).cuda() for a in (x, y, s))
    F = torch.empty((2 * clip.K + 1, 2 * clip.L + 1), dtype=torch.complex64, device="cuda")
    a = torch.empty(1, dtype=torch.int64, device="cuda")
    c = P._clip(x, y, s, x.numel(), clip.T, clip.K, clip.L, F, a)
    st = h.lib.fcfs_forward(h.ptr, ctypes.byref(c), P.PRECISIONS[prec], ctypes.c_void_p(ws),
                            ctypes.c_size_t(nbytes))
    return st, (x, y, s, F, a)


def test_short_and_misaligned_workspace(P):
    # FCFS_ERR_WORKSPACE (-5) before anything is enqueued, with a detail
    h = P.Handle()
    clip = synth.clip(81, 2048, 100, n_polygons=300)
    need = P.workspace_size(clip.n_vertices, clip.T, clip.K, clip.L, "bf16")
    buf = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    st, _ = _forward_call(P, h, clip, "bf16", buf.data_ptr(), need - 256)
    assert st == -5
    assert b"workspace too small" in h.lib.fcfs_last_error(h.ptr)
    st, _ = _forward_call(P, h, clip, "bf16", buf.data_ptr() + 64, need)
    assert st == -5
    assert b"aligned" in h.lib.fcfs_last_error(h.ptr)
    st, _ = _forward_call(P, h, clip, "bf16", None, need)
    assert st == -5
    # the exact size works and the handle is usable after the refusals
    st, keep = _forward_call(P, h, clip, "bf16", buf.data_ptr(), need)
    assert st == 0
    torch.cuda.synchronize()
    Fh = keep[3].cpu().numpy()
    Fr, _ = P.forward(*keep[:3], clip.T, clip.K, clip.L, precision="bf16", handle=h)
    torch.cuda.synchronize()
    assert np.array_equal(Fh, Fr.cpu().numpy())
    h.close()


def test_external_capture_is_refused(P):
    # a stream the caller is capturing into a graph is refused with
    # FCFS_ERR_UNSUPPORTED (-4) before the library enqueues anything
    clip = synth.clip(82, 1024, 40, n_polygons=50)
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    x, y, s = (torch.as_tensor(a).cuda() for a in (x, y, s))
    h = P.Handle()
    F0, _ = P.forward(x, y, s, clip.T, clip.K, clip.L, precision="bf16", handle=h)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    z = torch.zeros(8, device="cuda")
    with pytest.raises(P.FcfsError) as ei:
        with torch.cuda.graph(g):
            z.add_(1.0)
            P.forward(x, y, s, clip.T, clip.K, clip.L, precision="bf16", handle=h)
    assert ei.value.status == -4
    # outside the capture the handle works as before
    F1, _ = P.forward(x, y, s, clip.T, clip.K, clip.L, precision="bf16", handle=h)
    torch.cuda.synchronize()
    assert torch.equal(F0, F1)
    h.close()


def test_stream_switch_orders_the_handle(P):
    # One handle and one workspace, calls alternating between two streams with
    # no wait by the caller: a large clip on the first stream, then small ones
    # on the second and the first again.  The switch orders the new stream
    # after the old one, so every result equals the same call made alone (the
    # kernels are deterministic), bit for bit.
    big = synth.clip(84, 8192, 511, n_polygons=4000)
    small = synth.clip(85, 2048, 100, n_polygons=200)
    h = P.Handle()
    ins = []
    for c in (big, small):
        x, y, s, _, _ = P.loops_to_corners(c.xy, c.off)
        ins.append(tuple(torch.as_tensor(a).cuda() for a in (x, y, s)) + (c,))
    need = max(P.workspace_size(t[0].numel(), t[3].T, t[3].K, t[3].L, "bf16") for t in ins)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    out = [torch.empty((2 * t[3].K + 1, 2 * t[3].L + 1), dtype=torch.complex64, device="cuda")
           for t in (ins[0], ins[1], ins[1], ins[0])]
    area = torch.empty(4, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()

    def call(i, t, stream):
        P.check(h.lib.fcfs_set_stream(h.ptr, ctypes.c_void_p(stream.cuda_stream)), h.ptr)
        x, y, s, c = t
        cl = P._clip(x, y, s, x.numel(), c.T, c.K, c.L, out[i], area[i:i + 1])
        P.check(h.lib.fcfs_forward(h.ptr, ctypes.byref(cl), P.PRECISIONS["bf16"],
                                   ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(need)), h.ptr)

    _say("stream switch: big on s1, small on s2, small on s1, big on s2")
    for i, (t, st) in enumerate(((ins[0], s1), (ins[1], s2), (ins[1], s1), (ins[0], s2))):
        call(i, t, st)
    torch.cuda.synchronize()
    got = [o.clone() for o in out]
    for i, t in enumerate((ins[0], ins[1], ins[1], ins[0])):
        call(i, t, s1)
        torch.cuda.synchronize()
        assert torch.equal(got[i], out[i]), i
    # the binding: its cached workspace grows on one stream while the other
    # stream's call may still read the old one
    h2 = P.Handle()
    res = []
    for t, st in ((ins[1], s1), (ins[0], s2), (ins[1], s1)):
        x, y, s, c = t
        with torch.cuda.stream(st):
            res.append(P.forward(x, y, s, c.T, c.K, c.L, precision="bf16", handle=h2)[0])
    torch.cuda.synchronize()
    assert torch.equal(res[0], got[1]) and torch.equal(res[2], got[1])
    assert torch.equal(res[1], got[0])
    h2.close()
    h.close()


def _gclip(P, seed, Nx, Ny, F, K, n):
    # n polygons drawn on the grid of step 2^-F inside an Nx x Ny tile
    c = synth.clip(seed, min(Nx, Ny) << F, K, n_polygons=n)
    x, y, s, _, _ = P.loops_to_corners(c.xy, c.off)
    return (x, y, s, Nx, Ny, K, K, F), c


def test_plan_outlives_its_handle(P):
    # destroying the handle first detaches its captured plans; the plan is
    # then destroyed without touching the handle
    h = P.Handle()
    clips = [_gclip(P, 83 + i, 600 + 50 * i, 500, 1, 20, 20)[0] for i in range(3)]
    b = P.GeneralBatch(clips, precision="bf16", handle=h)
    torch.cuda.synchronize()
    b.run()
    torch.cuda.synchronize()
    h.close()
    b.close()
    # a new handle and plan work normally afterwards
    h2 = P.Handle()
    b2 = P.GeneralBatch(clips, precision="bf16", handle=h2)
    b2.run()
    torch.cuda.synchronize()
    b2.close()
    h2.close()


def test_general_batch_past_the_table_cache(P, oracle_lib):
    # 20 clips with 20 distinct x periods (the handle caches 16 period tables
    # and grows past that for tables a plan pins); then corners rewritten in
    # place between replays: every replay recomputes from the current corners
    h = P.Handle()
    specs = [(1000 + 37 * i, 1000, 0, 12, 30, 900 + i) for i in range(20)]
    clips, loops = [], []
    for Nx, Ny, F, K, n, seed in specs:
        cl, c = _gclip(P, seed, Nx, Ny, F, K, n)
        clips.append(cl)
        loops.append(c)
    b = P.GeneralBatch(clips, precision="bf16", handle=h)
    torch.cuda.synchronize()
    for i, (Nx, Ny, F, K, n, seed) in enumerate(specs):
        ref, area = oracle_lib.cfs_grid_general(loops[i].xy, loops[i].off, Nx, Ny, K, K)
        e = float(np.max(np.abs(b.F[i].cpu().numpy().astype(np.complex128) - ref)) / abs(ref[K, K]))
        assert int(b.area[i].item()) == area
        assert e <= TOL_SPLIT, (i, e)
    # rewrite the corners of every clip (same count: the polygons shifted by
    # one grid step along x) and replay twice
    for rep in range(2):
        for i, (x, y, s) in enumerate(b.corners):
            x.add_(1)
        b.run()
        torch.cuda.synchronize()
        for i, (Nx, Ny, F, K, n, seed) in enumerate(specs):
            xy = loops[i].xy.astype(np.int64) + np.array([rep + 1, 0])
            x, y, s = (t.clone() for t in b.corners[i])
            Fs, a = P.forward_general(x, y, s, Nx, Ny, K, K, frac_bits=F, precision="bf16",
                                      handle=h)
            torch.cuda.synchronize()
            # the batch sums in its own split order: agreement to the
            # precision's bound (a stale replay misses by orders more)
            f00 = abs(complex(Fs[K, K].item()))
            d = float(np.max(np.abs(Fs.cpu().numpy().astype(np.complex128)
                                    - b.F[i].cpu().numpy())) / f00)
            assert d <= TOL_SPLIT, (rep, i, d)
            if i % 7 == 0:
                ref, area = oracle_lib.cfs_grid_general(xy, loops[i].off, Nx, Ny, K, K)
                e = float(np.max(np.abs(Fs.cpu().numpy().astype(np.complex128) - ref))
                          / abs(ref[K, K]))
                assert e <= TOL_SPLIT, (rep, i, e)
    _say(f"general batch of {len(specs)} clips, {len(set(s[0] for s in specs))} periods: ok")
    b.close()
    h.close()
