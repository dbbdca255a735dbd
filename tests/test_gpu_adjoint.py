"""GPU parity of the adjoint (edge-offset gradient) against the FP64 oracle.

The oracle's analytic gradient is itself pinned to central finite differences
(test_oracle_pins).  Tolerances relative to max |g|: FP32 contraction 1e-5,
split-bf16 / split-fp16 1e-4.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GTOL = {"fp32": 1e-5, "bf16": 1e-4, "fp16": 1e-4}


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_5562_amd as P

    torch.cuda.set_device(0)
    return P


def _say(msg):
    print(msg, flush=True)


def _gpu_edge_grad(P, clip, G, prec, band=None):
    x, y, s, he, ve = P.loops_to_corners(clip.xy, clip.off)
    Gd = torch.as_tensor(G.astype(np.complex64)).cuda()
    gx, gy = P.adjoint(x, y, s, clip.T, clip.K, clip.L, Gd, precision=prec, band=band)
    ge = P.edge_grad(gx, gy, he, ve, x.size)
    torch.cuda.synchronize()
    return ge.cpu().numpy().astype(np.float64)


def _rand_G(K, L, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(2 * K + 1, 2 * L + 1)) + 1j * rng.normal(size=(2 * K + 1, 2 * L + 1))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_adjoint_random_cotangent(P, oracle_lib, prec):
    # a linear loss Re sum conj(G) F with a dense random G: every (k, l),
    # axes and DC included; K != L, several GEMM column groups, ragged corners
    T, K, L = 512, 37, 150
    clip = synth.clip(41, T, K, L, n_polygons=40)
    _say(f"adjoint V={clip.n_vertices} T={T} K={K} L={L} prec={prec}")
    G = _rand_G(K, L, 1)
    want = oracle_lib.edge_grad(clip.xy, clip.off, T, K, L, G.astype(np.complex64))
    got = _gpu_edge_grad(P, clip, G, prec)
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    _say(f"  err/max|g| = {e:.3e}")
    assert e <= GTOL[prec]


@pytest.mark.parametrize("K,L", [(25, 110), (120, 80)])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_adjoint_register_resident_step_counts(P, oracle_lib, K, L, prec):
    # the register-resident main term for k bands of 32 and 128 rows (two and
    # eight 16-row steps per column block, three and two chunks of 32
    # frequencies per set), with chunk counts (4 and 3) that leave a partial
    # set
    T = 1024
    clip = synth.clip(43, T, K, L, n_polygons=40)
    _say(f"adjoint V={clip.n_vertices} T={T} K={K} L={L} prec={prec}")
    G = _rand_G(K, L, 3)
    want = oracle_lib.edge_grad(clip.xy, clip.off, T, K, L, G.astype(np.complex64))
    got = _gpu_edge_grad(P, clip, G, prec)
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    _say(f"  err/max|g| = {e:.3e}")
    assert e <= GTOL[prec]


def test_adjoint_band_matches_full(P):
    T, K, L = 1024, 64, 64
    clip = synth.clip(42, T, K, L, n_polygons=60)
    G = _rand_G(K, L, 2)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-L, L + 1), indexing="ij")
    G[(kk**2 + ll**2) > 20**2] = 0
    full = _gpu_edge_grad(P, clip, G, "fp32")
    band = _gpu_edge_grad(P, clip, G, "fp32", band=(20, 20))
    assert np.max(np.abs(full - band)) <= 1e-5 * np.max(np.abs(full))


def _pupil(K, L, r):
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-L, L + 1), indexing="ij")
    return (kk**2 + ll**2 <= r * r).astype(np.float64)


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_pupil_loss_gradient(P, oracle_lib, prec):
    # L = sum |H F - G_t|^2, H a circular pupil of radius 0.35 K, G_t the
    # pupil-filtered spectrum of a second seeded clip (computed by the oracle).
    T, K = 4096, 255
    r = 0.35 * K
    rb = int(np.floor(r))
    clip = synth.clip(5, T, K, min_vertices=20_000)
    clip2 = synth.clip(6, T, K, min_vertices=20_000)
    _say(f"pupil loss V={clip.n_vertices} T={T} K={K} prec={prec}")
    Hp = _pupil(K, K, r)
    # oracle spectra on the band only (H is zero outside)
    kk, ll = np.nonzero(Hp)
    kb, lb = kk - K, ll - K
    Gt = np.zeros_like(Hp, dtype=np.complex128)
    Gt[kk, ll] = oracle_lib.cfs_points(clip2.xy, clip2.off, T, kb, lb)
    Gt = Gt.astype(np.complex64).astype(np.complex128)
    Fo = np.zeros_like(Gt)
    Fo[kk, ll] = oracle_lib.cfs_points(clip.xy, clip.off, T, kb, lb)
    Go = 2 * Hp * (Hp * Fo - Gt)
    rng = np.random.default_rng(7)
    edges = rng.choice(clip.n_vertices, 256, replace=False)
    want = oracle_lib.edge_grad(clip.xy, clip.off, T, K, K, Go, edges=edges)
    # GPU: forward, cotangent from the loss, adjoint restricted to the pupil band
    x, y, s, he, ve = P.loops_to_corners(clip.xy, clip.off)
    F, _ = P.forward(x, y, s, T, K, K, precision=prec)
    Hd = torch.as_tensor(Hp, dtype=torch.float32).cuda()
    Gtd = torch.as_tensor(Gt.astype(np.complex64)).cuda()
    Gd = 2 * Hd * (Hd * F - Gtd)
    gx, gy = P.adjoint(x, y, s, T, K, K, Gd, precision=prec, band=(rb, rb))
    ge = P.edge_grad(gx, gy, he, ve, x.size).cpu().numpy().astype(np.float64)
    e = float(np.max(np.abs(ge[edges] - want)) / np.max(np.abs(want)))
    _say(f"  err/max|g| over {edges.size} edges = {e:.3e}")
    assert e <= GTOL[prec]


def test_autograd_function(P, oracle_lib):
    T, K = 256, 24
    clip = synth.clip(43, T, K, n_polygons=12)
    geom = P.Geometry(clip.xy, clip.off, T, K)
    off = torch.zeros(geom.n_edges, dtype=torch.float32, device="cuda", requires_grad=True)
    F = P.FCFSFunction.apply(off, geom, "fp32")
    Hp = torch.as_tensor(_pupil(K, K, 0.35 * K), dtype=torch.float32).cuda()
    loss = ((Hp * F).abs() ** 2).sum()
    loss.backward()
    Fo, _ = oracle_lib.cfs_grid(clip.xy, clip.off, T, K, K)
    Hn = _pupil(K, K, 0.35 * K)
    want = oracle_lib.edge_grad(clip.xy, clip.off, T, K, K, 2 * Hn * Hn * Fo)
    got = off.grad.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want))
    # an integer shift of the edges moves the corners accordingly
    shift = torch.zeros(geom.n_edges, device="cuda")
    shift[0] = 3.0
    x, y = geom.corners(shift)
    assert int((x.cpu() - geom.base_x.cpu()).abs().sum() + (y.cpu() - geom.base_y.cpu()).abs().sum()) == 6
    with pytest.raises(P.FcfsError):
        geom.corners(shift + 0.5)
    # without the check, offsets are rounded to the nearest integer (ties to even)
    lax = P.Geometry(clip.xy, clip.off, T, K, check_offsets=False)
    frac = torch.zeros(geom.n_edges, device="cuda")
    frac[0], frac[1], frac[2], frac[3] = 2.6, -1.4, 0.5, 1.5
    xr, yr = lax.corners(frac)
    xw, yw = geom.corners(torch.round(frac))
    assert torch.equal(xr, xw) and torch.equal(yr, yw)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_autograd_low_pass(P, oracle_lib, prec):
    # FCFSFunction with a band and a disc: F is the low-pass spectrum M F and
    # the gradient of sum |M F|^2 is the adjoint of M (2 M F)
    T, K = 512, 40
    r = 17.5
    clip = synth.clip(44, T, K, n_polygons=30)
    geom = P.Geometry(clip.xy, clip.off, T, K)
    off = torch.zeros(geom.n_edges, dtype=torch.float32, device="cuda", requires_grad=True)
    F = P.FCFSFunction.apply(off, geom, prec, (20, 20), r)
    loss = (F.abs() ** 2).sum()
    loss.backward()
    Fo, _ = oracle_lib.cfs_grid(clip.xy, clip.off, T, K, K)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    M = ((kk ** 2 + ll ** 2 <= r * r) & (np.abs(kk) <= 20) & (np.abs(ll) <= 20)).astype(np.float64)
    Fm = F.detach().cpu().numpy().astype(np.complex128)
    assert np.all(Fm[M == 0] == 0)
    assert np.max(np.abs(Fm - M * Fo)) <= (1e-6 if prec == "fp32" else 1e-5) * abs(Fo[K, K])
    want = oracle_lib.edge_grad(clip.xy, clip.off, T, K, K, 2 * M * Fo)
    got = off.grad.cpu().numpy().astype(np.float64)
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    _say(f"low-pass autograd {prec}: err/max|g| = {e:.3e}")
    assert e <= GTOL[prec]


def test_pupil_loss_kernel(P):
    # value and cotangent of sum |H F - G|^2 against the same arithmetic in
    # numpy FP64, for the disc mask and for explicit weights
    rng = np.random.default_rng(11)
    K, L = 70, 45
    F = (rng.normal(size=(2 * K + 1, 2 * L + 1)) + 1j * rng.normal(size=(2 * K + 1, 2 * L + 1))).astype(np.complex64)
    G = (rng.normal(size=F.shape) + 1j * rng.normal(size=F.shape)).astype(np.complex64)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-L, L + 1), indexing="ij")
    for H, radius in ((None, 30.5), (rng.uniform(0, 2, F.shape).astype(np.float32), None)):
        Ft = torch.as_tensor(F).cuda().requires_grad_(True)
        Gt = torch.as_tensor(G).cuda()
        loss = P.PupilLoss.apply(Ft, Gt, radius, None if H is None else torch.as_tensor(H).cuda())
        loss.backward()
        torch.cuda.synchronize()
        h = (kk ** 2 + ll ** 2 <= radius ** 2).astype(np.float64) if H is None else H.astype(np.float64)
        d = h * F.astype(np.complex128) - G.astype(np.complex128)
        want = float(np.sum(np.abs(d) ** 2))
        assert abs(float(loss.item()) - want) <= 1e-12 * want
        gw = (2 * h * d)
        got = Ft.grad.cpu().numpy()
        assert np.array_equal(got.real, gw.real.astype(np.float32))
        assert np.array_equal(got.imag, gw.imag.astype(np.float32))


def test_pupil_loss_in_the_optimisation_step(P):
    # the fused loss gives the same edge gradient as the loss written in torch ops
    T, K = 1024, 40
    r = 0.35 * K
    rb = int(np.floor(r))
    clip = synth.clip(43, T, K, n_polygons=50)
    geom = P.Geometry(clip.xy, clip.off, T, K)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    Hd = torch.as_tensor((kk ** 2 + ll ** 2 <= r * r).astype(np.float32)).cuda()
    rng = np.random.default_rng(3)
    Gt = Hd * torch.as_tensor((rng.normal(size=kk.shape) + 1j * rng.normal(size=kk.shape)).astype(np.complex64)).cuda()
    grads = []
    for fused in (False, True):
        off = torch.zeros(geom.n_edges, dtype=torch.float32, device="cuda", requires_grad=True)
        Fv = P.FCFSFunction.apply(off, geom, "fp32", (rb, rb), r)
        loss = P.PupilLoss.apply(Fv, Gt, r) if fused else ((Hd * Fv - Gt).abs() ** 2).sum()
        loss.backward()
        grads.append(off.grad.cpu().numpy().astype(np.float64))
    assert np.max(np.abs(grads[0] - grads[1])) <= 1e-5 * np.max(np.abs(grads[0]))


@pytest.mark.skip(reason="capturing the autograd step with torch.cuda.graph ended in a "
                         "segmentation fault inside the HIP runtime at capture end (cause not "
                         "identified); the library now refuses a stream the caller is capturing "
                         "(FCFS_ERR_UNSUPPORTED, test_gpu_boundary.py::"
                         "test_external_capture_is_refused) and captures the step itself "
                         "(fcfs_pupil_step_plan, tested replay by replay)")
def test_optimisation_step_in_a_graph(P):
    # The whole step (edge offsets -> low-pass forward -> fused loss ->
    # adjoint -> edge gradient) captured once in a graph and replayed: every
    # replay, with eager steps in between, reproduces the eager gradient bit
    # for bit (the kernels are deterministic).
    T, K = 1024, 40
    r = 0.35 * K
    rb = int(np.floor(r))
    clip = synth.clip(44, T, K, n_polygons=120)
    geom = P.Geometry(clip.xy, clip.off, T, K, check_offsets=False)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    Hd = torch.as_tensor((kk ** 2 + ll ** 2 <= r * r).astype(np.float32)).cuda()
    rng = np.random.default_rng(5)
    Gt = Hd * torch.as_tensor((rng.normal(size=kk.shape) + 1j * rng.normal(size=kk.shape)).astype(np.complex64)).cuda()
    offs = [torch.as_tensor(rng.integers(-2, 3, geom.n_edges).astype(np.float32)).cuda()
            for _ in range(2)]
    off = torch.zeros(geom.n_edges, dtype=torch.float32, device="cuda", requires_grad=True)

    def step():
        off.grad = None
        Fv = P.FCFSFunction.apply(off, geom, "bf16", (rb, rb), r)
        loss = P.PupilLoss.apply(Fv, Gt, r)
        loss.backward()
        return loss

    want = []
    for o in offs:
        with torch.no_grad():
            off.copy_(o)
        loss = step()
        want.append((off.grad.clone(), loss.detach().clone()))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    keep = P.default_handle()._ws  # the workspace the captured launches use
    graph = torch.cuda.CUDAGraph()
    off.grad = None
    with torch.cuda.graph(graph):
        loss_g = step()
    grad_g = off.grad
    for it in range(4):
        with torch.no_grad():
            off.copy_(offs[it % 2])
        graph.replay()
        torch.cuda.synchronize()
        _say(f"graph replay {it}")
        assert torch.equal(grad_g, want[it % 2][0])
        assert torch.equal(loss_g, want[it % 2][1])
        step()  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(off.grad, want[it % 2][0])
    del keep


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_pupil_step_matches_the_autograd_step(P, prec):
    # the one-call step enqueues the same launches as the autograd path:
    # loss, edge gradient and spectrum agree bit for bit (disc H and given H)
    T, K = 2048, 60
    r = 0.35 * K
    rb = int(np.floor(r))
    clip = synth.clip(45, T, K, n_polygons=150)
    geom = P.Geometry(clip.xy, clip.off, T, K, check_offsets=False)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    Hn = (kk ** 2 + ll ** 2 <= r * r).astype(np.float32)
    rng = np.random.default_rng(8)
    Gt = torch.as_tensor((Hn * (rng.normal(size=kk.shape) + 1j * rng.normal(size=kk.shape)))
                         .astype(np.complex64)).cuda()
    offs = torch.as_tensor(rng.integers(-3, 4, geom.n_edges).astype(np.float32)).cuda()
    for H in (None, torch.as_tensor(Hn * 0.5).cuda()):
        off = offs.clone().requires_grad_(True)
        Fv = P.FCFSFunction.apply(off, geom, prec, (rb, rb), r)
        loss = P.PupilLoss.apply(Fv, Gt, r, H)
        loss.backward()
        Fs = torch.empty_like(Fv)
        ls, gs = P.pupil_step(geom, offs, Gt, radius=r, band=(rb, rb), H=H, precision=prec,
                              F_out=Fs)
        torch.cuda.synchronize()
        assert torch.equal(Fs, Fv.detach())
        assert torch.equal(ls, loss.detach())
        assert torch.equal(gs, off.grad)
        _say(f"pupil step {prec} H={'disc' if H is None else 'weights'}: loss {float(ls):.6e}")


def test_pupil_step_plan_replays(P):
    # the captured step replayed with new offsets, eager work and
    # synchronisations in between: every replay equals the one-call step
    T, K = 2048, 60
    r = 0.35 * K
    rb = int(np.floor(r))
    clip = synth.clip(46, T, K, n_polygons=150)
    geom = P.Geometry(clip.xy, clip.off, T, K, check_offsets=False)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    Hn = (kk ** 2 + ll ** 2 <= r * r).astype(np.float32)
    rng = np.random.default_rng(9)
    Gt = torch.as_tensor((Hn * (rng.normal(size=kk.shape) + 1j * rng.normal(size=kk.shape)))
                         .astype(np.complex64)).cuda()
    offs = [torch.as_tensor(rng.integers(-3, 4, geom.n_edges).astype(np.float32)).cuda()
            for _ in range(3)]
    want = []
    for o in offs:
        Fw = torch.empty_like(Gt)
        lw, gw = P.pupil_step(geom, o, Gt, radius=r, band=(rb, rb), F_out=Fw)
        want.append((lw.clone(), gw.clone(), Fw))
    plan = P.PupilStep(geom, Gt, radius=r, band=(rb, rb))
    for it in range(6):
        i = it % 3
        loss, g = plan.run(offs[i])
        torch.cuda.synchronize()
        _say(f"step plan replay {it}")
        assert torch.equal(loss, want[i][0]) and torch.equal(g, want[i][1])
        assert torch.equal(plan.F, want[i][2])
        junk = torch.randn(1 << 18, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del junk
    plan.close()


def test_optimisation_step_full_size_sampled(P, oracle_lib):
    # the differentiation workload at full size: 100k corners, T = 4096,
    # |k|,|l| <= 255, pupil of radius 0.35 K, target the pupil-filtered
    # spectrum of a second clip (from the oracle); the one-call step's edge
    # gradient on 128 sampled edges against the oracle's analytic gradient
    T, K = 4096, 255
    r = 0.35 * K
    rb = int(np.floor(r))
    clip = synth.clip(5, T, K, min_vertices=100_000)
    clip2 = synth.clip(6, T, K, min_vertices=100_000)
    _say(f"full-size step V={clip.n_vertices} T={T} K={K}")
    Hp = _pupil(K, K, r)
    kk, ll = np.nonzero(Hp)
    Gt = np.zeros_like(Hp, dtype=np.complex128)
    Gt[kk, ll] = oracle_lib.cfs_points(clip2.xy, clip2.off, T, kk - K, ll - K)
    Gt = Gt.astype(np.complex64).astype(np.complex128)
    Fo = np.zeros_like(Gt)
    Fo[kk, ll] = oracle_lib.cfs_points(clip.xy, clip.off, T, kk - K, ll - K)
    rng = np.random.default_rng(12)
    edges = rng.choice(clip.n_vertices, 128, replace=False)
    want = oracle_lib.edge_grad(clip.xy, clip.off, T, K, K, 2 * Hp * (Hp * Fo - Gt), edges=edges)
    geom = P.Geometry(clip.xy, clip.off, T, K, check_offsets=False)
    off = torch.zeros(geom.n_edges, dtype=torch.float32, device="cuda")
    loss, g = P.pupil_step(geom, off, torch.as_tensor(Gt.astype(np.complex64)).cuda(), radius=r,
                           band=(rb, rb))
    torch.cuda.synchronize()
    got = g.cpu().numpy().astype(np.float64)[edges]
    e = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    lo = float(np.sum(np.abs(Hp * Fo - Gt) ** 2))
    _say(f"  err/max|g| over {edges.size} edges = {e:.3e}; loss rel err "
         f"{abs(float(loss) - lo) / lo:.2e}")
    assert e <= GTOL["bf16"]
    assert abs(float(loss) - lo) <= 1e-4 * lo


def test_gradient_against_central_differences_on_the_gpu(P, oracle_lib):
    # The adjoint's edge gradient against central differences of the loss
    # sum |H F - G|^2 behind a pupil of radius 0.35 K, both on the GPU.  An
    # edge moved by t changes F by the transform of the strip it sweeps, and
    # the corner form is linear in the corner list: that difference is the
    # forward transform of four corners (the moved ones with their signs, the
    # base ones with opposite signs), so L(t) - L(0) is formed from it and
    # from F at the base offsets without cancellation.  Richardson's
    # combination (4 D(1) - D(2)) / 3 of the central differences at t = +-1,
    # +-2 removes their h^2 term; the error left, of order (h w)^4 with
    # w <= 2 pi r / T, is measured by the same differences of the FP64
    # oracle against its analytic gradient.  The GPU comparison allows that
    # plus the adjoint's own bound (1e-5 FP32, 1e-4 split, of max |g|).
    T, K = 1024, 40
    r = 0.35 * K
    rb = int(np.floor(r))
    clip = synth.clip(61, T, K, n_polygons=60)
    geom = P.Geometry(clip.xy, clip.off, T, K)
    kk, ll = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    H = (kk ** 2 + ll ** 2 <= r * r).astype(np.float64)
    rng = np.random.default_rng(61)
    Gn = (H * (rng.normal(size=kk.shape) + 1j * rng.normal(size=kk.shape)) * 40.0).astype(np.complex64)
    G = torch.as_tensor(Gn).cuda()
    Gd = Gn.astype(np.complex128)
    x0, y0, s0, he, ve = P.loops_to_corners(clip.xy, clip.off)
    off = clip.off
    n = int(off[-1])
    loop = np.repeat(np.arange(off.size - 1), np.diff(off))
    idx = np.arange(n)
    nxt = np.where(idx + 1 == off[loop + 1], off[loop], idx + 1)
    prv = np.where(idx == off[loop], off[loop + 1] - 1, idx - 1)

    F0g, _ = P.forward_fft(x0, y0, s0, T, K, K)  # the base spectrum (FP64 lattice form)
    torch.cuda.synchronize()
    res0 = H * F0g.cpu().numpy().astype(np.complex128) - Gd

    def strip(e, t):
        # F(edge e moved by t) - F(base) from the four corners of the strip
        a, b = int(e), int(nxt[e])
        vert = clip.xy[a, 0] == clip.xy[b, 0]
        xs = np.array([x0[a], x0[b], x0[a], x0[b]], np.int32)
        ys = np.array([y0[a], y0[b], y0[a], y0[b]], np.int32)
        if vert:
            xs[:2] += int(t)
        else:
            ys[:2] += int(t)
        ss = np.array([s0[a], s0[b], -s0[a], -s0[b]], np.int8)
        F, _ = P.forward(xs, ys, ss, T, K, K, precision="fp32")
        torch.cuda.synchronize()
        return H * F.cpu().numpy().astype(np.complex128)

    def fd_gpu(e):
        d = []
        for h in (1, 2):
            dp, dm = strip(e, h), strip(e, -h)
            dl = np.sum(2 * np.real(np.conj(res0) * (dp - dm)) + np.abs(dp) ** 2 - np.abs(dm) ** 2)
            d.append(dl / (2 * h))
        return (4 * d[0] - d[1]) / 3

    xy0 = clip.xy.astype(np.float64)

    def fd_oracle(e):
        d = []
        for h in (1.0, 2.0):
            lv = []
            for t in (h, -h):
                o = np.zeros(n)
                o[e] = t
                xy = xy0.copy()
                xy[:, 0] += o[ve]
                xy[:, 1] += o[he]
                F = oracle_lib.cfs_grid(xy, clip.off, T, K, K, lattice=False)[0]
                lv.append(float(np.sum(np.abs(H * F - Gd) ** 2)))
            d.append((lv[0] - lv[1]) / (2 * h))
        return (4 * d[0] - d[1]) / 3

    # analytic FP64 gradient of the oracle at the base offsets
    F0 = oracle_lib.cfs_grid(xy0, clip.off, T, K, K)[0]
    g_or = oracle_lib.edge_grad(clip.xy, clip.off, T, K, K, 2 * H * (H * F0 - Gd))
    # edges whose neighbours are at least 3 units long (moves of +-2 keep
    # every edge of the loop non-degenerate) and whose gradient is not tiny
    elen = np.abs(clip.xy[nxt] - clip.xy[idx]).sum(axis=1)
    ok = (elen[prv] >= 3) & (elen[nxt] >= 3) & (np.abs(g_or) > 1e-2 * np.max(np.abs(g_or)))
    edges = rng.choice(np.nonzero(ok)[0], 10, replace=False)
    gmax = float(np.max(np.abs(g_or)))
    fd_or = np.array([fd_oracle(e) for e in edges])
    fd_err = float(np.max(np.abs(fd_or - g_or[edges])) / gmax)
    fd_g = np.array([fd_gpu(e) for e in edges])
    _say(f"central differences: oracle FD vs analytic {fd_err:.2e}, GPU FD vs oracle FD "
         f"{np.max(np.abs(fd_g - fd_or)) / gmax:.2e} (of max |g|)")
    for prec, tol in (("fp32", 1e-5), ("bf16", 1e-4)):
        offt = torch.zeros(geom.n_edges, dtype=torch.float32, device="cuda", requires_grad=True)
        Fv = P.FCFSFunction.apply(offt, geom, prec, (rb, rb), r)
        loss = P.PupilLoss.apply(Fv, G, r)
        loss.backward()
        g = offt.grad.cpu().numpy().astype(np.float64)[edges]
        e = float(np.max(np.abs(g - fd_g)) / gmax)
        _say(f"  {prec}: adjoint vs GPU central differences: {e:.2e} of max |g|")
        assert e <= tol + 2 * fd_err + 1e-6
