"""Batched form: persistent graph-captured launch over clips of mixed sizes,
checked against the FP64 oracle and against the single-clip path; graph
replays; the autotuner and its cache."""
import json

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


def _clips(n, seed, v_hi=20_000):
    return synth.batch_clips(seed, n_clips=n, v_lo=1000, v_hi=v_hi, pool=256)


def _as_args(P, clips):
    out = []
    for c in clips:
        x, y, s, _, _ = P.loops_to_corners(c.xy, c.off)
        out.append((x, y, s, c.T, c.K, c.L))
    return out


def _sample(K, n, seed):
    rng = np.random.default_rng(seed)
    lo = np.array([(k, l) for k in range(-4, 5) for l in range(-4, 5)])
    kk = np.concatenate([lo[:, 0], rng.integers(-K, K + 1, n)])
    ll = np.concatenate([lo[:, 1], rng.integers(-K, K + 1, n)])
    return kk, ll


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp16"])
def test_batch_matches_oracle(P, oracle_lib, prec):
    clips = _clips(10, 5)
    _say(f"batch of {len(clips)} clips, V = {[c.n_vertices for c in clips]} prec={prec}")
    b = P.Batch(_as_args(P, clips), precision=prec)
    F = b.run()
    torch.cuda.synchronize()
    for i, c in enumerate(clips):
        kk, ll = _sample(c.K, 60, i)
        ref = oracle_lib.cfs_points(c.xy, c.off, c.T, kk, ll)
        f00 = abs(oracle_lib.cfs_points(c.xy, c.off, c.T, [0], [0])[0])
        got = F[i].cpu().numpy()[kk + c.K, ll + c.L]
        e = float(np.max(np.abs(got - ref)) / f00)
        _, area = oracle_lib.cfs_grid(c.xy, c.off, c.T, 0, 0)
        assert int(b.area[i].item()) == area
        assert e <= TOL[prec], (i, c.T, c.K, e)
    b.close()


def test_batch_low_fill_clips_near_axes(P, oracle_lib):
    # low-fill clips (disjoint cells) beside a dense one in one batch: every
    # coefficient with |k l| <= 160 meets the split bound, so the guard region
    # of each clip widened by itself; two replays give the same values
    cs = [synth.clip(22, 4096, 255, n_polygons=2000, disjoint=True),
          synth.clip(41, 2048, 127, n_polygons=300, disjoint=True),
          synth.clip(3, 1024, 63, n_polygons=400)]
    _say(f"low-fill batch V = {[c.n_vertices for c in cs]}")
    b = P.Batch(_as_args(P, cs), precision="bf16")
    F1 = [f.cpu().numpy().copy() for f in b.run()]
    F2 = [f.cpu().numpy() for f in b.run()]
    for i, c in enumerate(cs):
        pts = [(k, l) for k in range(-c.K, c.K + 1) for l in range(-c.L, c.L + 1)
               if k and l and abs(k * l) <= 160]
        kk, ll = np.array(pts).T
        ref = oracle_lib.cfs_points(c.xy, c.off, c.T, kk, ll)
        f00 = abs(oracle_lib.cfs_points(c.xy, c.off, c.T, [0], [0])[0])
        e = np.abs(F1[i][kk + c.K, ll + c.L] - ref) / f00
        w = int(np.argmax(e))
        _say(f"  clip {i}: max err/|F00| = {e[w]:.3e} at ({kk[w]},{ll[w]})")
        assert e[w] <= TOL["bf16"], (i, e[w])
        assert np.array_equal(F1[i], F2[i])
    b.close()


def test_batch_equals_single_clip_and_replays(P):
    clips = _clips(8, 6)
    args = _as_args(P, clips)
    b = P.Batch(args, precision="bf16")
    F1 = [f.cpu().numpy().copy() for f in b.run()]
    for i, (x, y, s, T, K, L) in enumerate(args):
        Fs, _ = P.forward(x, y, s, T, K, L, precision="bf16")
        d = np.max(np.abs(Fs.cpu().numpy() - F1[i])) / abs(F1[i][K, L])
        assert d <= 2e-6, (i, d)
    # replays, with eager work and synchronisations in between, give the same bits
    for r in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for f in b.F:
            f.zero_()
        F2 = [f.cpu().numpy() for f in b.run()]
        for i in range(len(F1)):
            assert np.array_equal(F1[i], F2[i]), (r, i)
        del junk
    # a plan built for other clips is refused
    other = P.Batch(args[:3], precision="bf16")
    other._plan = b._plan
    with pytest.raises(P.FcfsError):
        other.run()
    other._plan = type(other._plan)()
    b.close()


def test_batch_single_split_clips_write_directly(P, oracle_lib):
    # clips contracted in one split unfold their sums into F in the work item
    # itself (no partials); small bands inside the FP64 guard block, one-sided
    # bands and a multi-split clip ride in the same batch
    base = synth.clip(71, 2048, 127, n_polygons=120)
    big = synth.clip(72, 4096, 63, min_vertices=40_000)
    spec = [(base, 2048, 5, 5), (base, 2048, 0, 7), (base, 2048, 9, 0), (base, 2048, 20, 3),
            (base, 2048, 127, 127), (big, 4096, 63, 63)]
    args = []
    for c, T, K, L in spec:
        x, y, s, _, _ = P.loops_to_corners(c.xy, c.off)
        args.append((x, y, s, T, K, L))
    _say(f"single-split batch: V = {[a[0].size for a in args]}")
    b = P.Batch(args, precision="bf16")
    F = [f.cpu().numpy().astype(np.complex128) for f in b.run()]
    torch.cuda.synchronize()
    for i, (c, T, K, L) in enumerate(spec):
        ref, area = oracle_lib.cfs_grid(c.xy, c.off, T, K, L) if c is base else (None, None)
        if ref is None:
            kk, ll = _sample(K, 80, i)
            refp = oracle_lib.cfs_points(c.xy, c.off, T, kk, ll)
            f00 = abs(oracle_lib.cfs_points(c.xy, c.off, T, [0], [0])[0])
            e = float(np.max(np.abs(F[i][kk + K, ll + L] - refp)) / f00)
        else:
            e = float(np.max(np.abs(F[i] - ref)) / abs(ref[K, L]))
            assert int(b.area[i].item()) == area
        _say(f"  clip {i} T={T} K={K} L={L}: err/|F00| = {e:.3e}")
        assert e <= TOL["bf16"], (i, e)
    b.close()


def test_autotune_and_cache(P, tmp_path):
    path = tmp_path / "tune.json"
    h = P.Handle()
    P.autotune(path, effort=0, handle=h)
    doc = json.loads(path.read_text())
    assert doc["format"] == "fcfs-autotune-1"
    assert doc["forward"] and doc["batch"]
    # a fresh handle reads the cache; a malformed one is refused and ignored
    h2 = P.Handle()
    P.load_tune(path, handle=h2)
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    with pytest.raises(P.FcfsError):
        P.load_tune(bad, handle=h2)
    clip, _, _ = synth.clip_c1(1)
    x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    Fa, _ = P.forward(x, y, s, clip.T, clip.K, clip.L, precision="bf16", handle=h2)
    Fb, _ = P.forward(x, y, s, clip.T, clip.K, clip.L, precision="bf16", handle=h)
    torch.cuda.synchronize()
    assert np.allclose(Fa.cpu().numpy(), Fb.cpu().numpy(), atol=1e-5 * abs(Fa[clip.K, clip.L].item()))


def test_batch_autotuner_on_its_clips(P):
    # the batch autotuner times candidate plans on the clips themselves; the
    # plan it leaves gives the same coefficients as the single-clip forward
    clips = _clips(9, 6)
    args = _as_args(P, clips)
    h = P.Handle()
    b = P.Batch(args, precision="bf16", handle=h, tune=True)
    assert set(b.choice) == {P.batch_kbucket(a[4], a[5]) for a in args}
    for tile, chunk in b.choice.values():
        assert tile in (3, 4, 5) and chunk in (8192, 16384, 32768, 65536)
    F = [f.cpu().numpy().copy() for f in b.run()]
    for i, (x, y, s, T, K, L) in enumerate(args):
        Fs, _ = P.forward(x, y, s, T, K, L, precision="bf16", handle=h)
        d = np.max(np.abs(Fs.cpu().numpy() - F[i])) / abs(F[i][K, L])
        assert d <= 2e-6, (i, d)
    b.close()


def test_batch_per_bucket_variants(P, oracle_lib, tmp_path):
    # per-K-bucket choices from a cache file: K <= 63 on the two-wave variant 3
    # with small work items, K <= 511 on the pipelined variant 5, K <= 255 on
    # variant 4: three persistent launches in one plan; every clip matches the
    # single-clip forward and the oracle, replays repeat the first run
    cache = {"format": "fcfs-autotune-1", "forward": [], "batch": [
        {"prec": 1, "kbucket": 0, "tile": 3, "chunk": 8192},
        {"prec": 1, "kbucket": 2, "tile": 4, "chunk": 32768},
        {"prec": 1, "kbucket": 3, "tile": 5, "chunk": 16384}]}
    path = tmp_path / "buckets.json"
    path.write_text(json.dumps(cache))
    h = P.Handle()
    P.load_tune(path, handle=h)
    specs = [(1024, 63, 3000), (8192, 511, 9000), (4096, 255, 20000), (1024, 63, 25000),
             (8192, 511, 1500)]
    clips = [synth.clip(400 + i, T, K, min_vertices=V) for i, (T, K, V) in enumerate(specs)]
    args = _as_args(P, clips)
    b = P.Batch(args, precision="bf16", handle=h)
    assert b.choice == {0: (3, 8192), 2: (4, 32768), 3: (5, 16384)}
    F1 = [f.cpu().numpy().copy() for f in b.run()]
    F2 = [f.cpu().numpy().copy() for f in b.run()]
    for i, (x, y, s, T, K, L) in enumerate(args):
        assert np.array_equal(F1[i], F2[i]), i
        Fs, _ = P.forward(x, y, s, T, K, L, precision="bf16", handle=h)
        d = np.max(np.abs(Fs.cpu().numpy() - F1[i])) / abs(F1[i][K, L])
        assert d <= 2e-6, (i, d)
        c = clips[i]
        kk, ll = _sample(K, 40, i)
        ref = oracle_lib.cfs_points(c.xy, c.off, T, kk, ll)
        f00 = abs(oracle_lib.cfs_points(c.xy, c.off, T, [0], [0])[0])
        e = float(np.max(np.abs(F1[i][kk + K, ll + L] - ref)) / f00)
        assert e <= TOL["bf16"], (i, e)
    b.close()


def test_batch_full_size_sampled(P, oracle_lib):
    # the batching workload at full size: 256 clips, corners log-uniform in
    # [1k, 200k], (T, K) over {(1024,63),(2048,127),(4096,255),(8192,511)};
    # sampled coefficients of the 4 smallest, 4 largest and 4 random clips
    clips = synth.batch_clips(4, n_clips=256)
    args = _as_args(P, clips)
    _say(f"full-size batch: {sum(a[0].size for a in args)} corners")
    b = P.Batch(args, precision="bf16")
    F = b.run()
    torch.cuda.synchronize()
    order = np.argsort([a[0].size for a in args])
    rng = np.random.default_rng(13)
    pick = list(order[:4]) + list(order[-4:]) + list(rng.choice(order[4:-4], 4, replace=False))
    for i in pick:
        c = clips[i]
        kk, ll = _sample(c.K, 40, int(i))
        ref = oracle_lib.cfs_points(c.xy, c.off, c.T, kk, ll)
        f00 = abs(oracle_lib.cfs_points(c.xy, c.off, c.T, [0], [0])[0])
        e = float(np.max(np.abs(F[i].cpu().numpy()[kk + c.K, ll + c.L] - ref)) / f00)
        _say(f"  clip {i}: V={c.n_vertices} T={c.T} K={c.K} err/|F00| = {e:.3e}")
        assert e <= TOL["bf16"], (i, e)
    b.close()
