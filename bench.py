#!/usr/bin/env python3
"""Throughput benchmark of the FCFS transforms on one MI355X.

Headline workload (the precision form): one synthetic layout clip of >= 200,000
corners (polygons of 1-10 merged rectangles of 20-400 units, seed 3), period
T = 8192, every coefficient |k|, |l| <= 511 (a 1023 x 1023 grid).  One step =
one full forward pass (pre-pass, FP64 axis sums, MFMA contraction, epilogue)
on corners already resident in HBM, contraction in split-bf16.  The same clip
is also run with the FP32 contraction (the comparison form) and split-fp16.

Further forms, reported beside the headline:
  layout clip   2,000 polygons, T = 4096, |k|,|l| <= 255, FP32 and split-bf16
  lattice form  the FP64 lattice (FFT) form on the precision and layout clips
  general tile  the precision clip on an 8000 x 6000 tile, the layout clip on
                half units over 4000 x 3000 (periods not powers of two)
  pcht          the pruned continuous Haar transform of the layout clip, 12
                levels over its 4096 tile, bit-exact against the oracle
  single        one 64-corner polygon, T = 2048, |k|,|l| <= 64: microseconds
                per direct call and per one-clip graph replay
  batch         256 clips, corners log-uniform in [1k, 200k], (T, K) in
                {(1024,63), (2048,127), (4096,255), (8192,511)}, one replayed
                graph, split-bf16
  adjoint       100k corners, T = 4096, K = 255, pupil loss (radius 0.35 K):
                forward + backward (edge-offset gradient), split-bf16

Metric: vertex-coefficient pairs per second, V (2K+1)(2L+1) / time per step.
Printed as one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vertex·coefficient pairs/s: split-BF16 MFMA FCFS vs FP32 plain at ≤1e-5 rel err"
PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}  # MI355X dense MFMA
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "contract_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1010_5562_amd", "csrc", "fcfs_kernels.hip")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(key: str):
    """HBM bytes per contraction launch from the committed rocprofv3 counter
    runs, or None when the kernel source changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    e = t.get("entries", {}).get(key)
    return None if e is None else e.get("bytes_per_launch")


def timed(fn, steps: int, warmup: int, handle, kinds=("contract",)):
    """Runs fn warmup + steps times; returns (ms per step, per-kernel events).

    Only the launches of ``kinds`` are bracketed by events inside the timed
    region (two event records per launch on the launch's own stream); with
    kinds None nothing is."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if kinds is not None:
        handle.profile_begin(kinds)
    t_a = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    prof = handle.profile_end() if kinds is not None else None
    return (t_b - t_a) * 1e3 / steps, prof


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else None}


def streaming_gbps(P, V, T, K, L, breakdown):
    info = P.plan_info(V, T, K, L, "bf16")
    vpad = info["nsplit"] * info["chunk"]
    pre_bytes = 9 * V + 16 * vpad
    epi_bytes = 16 * info["nsplit"] * K * L + 8 * (2 * K + 1) * (2 * L + 1)
    out = {"plan": info, "prepass_bytes": pre_bytes, "epilogue_bytes": epi_bytes}
    if breakdown.get("prepass"):
        out["prepass"] = pre_bytes / (breakdown["prepass"] * 1e-3) / 1e9
    if breakdown.get("epilogue"):
        out["epilogue"] = epi_bytes / (breakdown["epilogue"] * 1e-3) / 1e9
    return out


def step_stats(fn, n: int):
    """Per-step device time of n further steps, each bracketed by events on
    the current stream (every kernel of a step, side stream included, ends
    before the step's last launch): mean with its 95% confidence half-width,
    median, min and max in ms."""
    import numpy as np
    import torch

    evs = []
    for _ in range(n):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return {"n": n, "mean": float(t.mean()),
            "ci95": float(1.96 * t.std(ddof=1) / np.sqrt(n)) if n > 1 else None,
            "median": float(np.median(t)), "min": float(t.min()), "max": float(t.max())}


def breakdown(fn, steps: int, handle):
    """Per-kind average kernel times from extra, untimed steps with events
    around every launch."""
    import torch

    torch.cuda.synchronize()
    handle.profile_begin()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    prof = handle.profile_end()
    return {k: kavg(prof, k) for k in ("prepass", "axis", "contract", "epilogue")}


def kavg(prof, kind):
    ms, n = prof[kind]
    return ms / n if n else None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="headline leg only (split-bf16 on the precision clip)")
    ap.add_argument("--check-adjoint", action="store_true",
                    help="also check the adjoint form's gradient against the oracle (slow)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter "
                         "calibration for rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 3}))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the library has no "
              "multi-GPU path.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1010_5562_amd as P
    import synth

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    h = P.default_handle()

    # ------------------------------------------------------------------ C3
    T, K = 8192, 511
    L = K
    t0 = time.time()
    clip = synth.clip(3, T, K, min_vertices=200_000)
    # canonicalisation (host, outside the timed region): loops -> signed corner
    # list and edge maps, timed on its own
    tc = time.perf_counter()
    for _ in range(5):
        x, y, s, _, _ = P.loops_to_corners(clip.xy, clip.off)
    canon_ms = (time.perf_counter() - tc) / 5 * 1e3
    V = int(x.size)
    pairs = V * (2 * K + 1) * (2 * L + 1)
    log(f"precision clip V={V} polygons={clip.n_loops} T={T} K={K} "
        f"(generated in {time.time() - t0:.1f}s)")
    xd, yd, sd = (torch.as_tensor(a).to(dev) for a in (x, y, s))
    F = torch.empty((2 * K + 1, 2 * L + 1), dtype=torch.complex64, device=dev)
    area = torch.empty(1, dtype=torch.int64, device=dev)

    legs = {}
    for prec in (["bf16"] if args.quick else ["bf16", "fp32", "fp16"]):
        ms, prof = timed(lambda: P.forward(xd, yd, sd, T, K, L, precision=prec, out=F,
                                           area_out=area), args.steps, args.warmup, h)
        legs[prec] = {"ms": ms, "prof": prof, "F": F.cpu().numpy().astype(np.complex128),
                      "area": int(area.item())}
        if prec == "bf16":
            legs[prec]["breakdown"] = breakdown(
                lambda: P.forward(xd, yd, sd, T, K, L, precision=prec, out=F, area_out=area),
                max(3, args.steps // 2), h)
            legs[prec]["stats"] = step_stats(
                lambda: P.forward(xd, yd, sd, T, K, L, precision=prec, out=F, area_out=area), 10)
        log(f"{prec}: {ms:.3f} ms/step  {pairs / ms * 1e3:.4g} pairs/s  "
            f"contract {kavg(prof, 'contract'):.3f} ms")

    # Oracle sample: the low-frequency block |k|,|l| <= 8 (where the 1/(k l)
    # weight concentrates the error) plus random (k, l); it serves both the
    # error report and the CPU baseline timing.
    import oracle

    cores = oracle.threads(0)
    rng = np.random.default_rng(12345)
    lo = np.array([(k, l) for k in range(-8, 9) for l in range(-8, 9)])
    # plus the strips next to the axes (one index small, the other anywhere),
    # where alpha_{k,l} ~ 1/(k l) is still large
    nst = 200
    ks = rng.choice(np.r_[-16:0, 1:17], nst)
    lr = rng.integers(-L, L + 1, nst)
    kk = np.concatenate([lo[:, 0], ks, rng.integers(-K, K + 1, nst)])
    ll = np.concatenate([lo[:, 1], lr, rng.choice(np.r_[-16:0, 1:17], nst)])
    tc = time.perf_counter()
    ref = oracle.cfs_points(clip.xy, clip.off, T, kk, ll)
    t_pts = time.perf_counter() - tc
    cpu = None
    if not args.no_cpu_baseline:
        budget = max(0.0, args.cpu_seconds - t_pts)
        n_more = int(budget / max(t_pts / kk.size, 1e-9))
        if n_more > 0:
            rk = rng.integers(-K, K + 1, n_more)
            rl = rng.integers(-L, L + 1, n_more)
            tc = time.perf_counter()
            ref2 = oracle.cfs_points(clip.xy, clip.off, T, rk, rl)
            t_pts += time.perf_counter() - tc
            kk, ll = np.concatenate([kk, rk]), np.concatenate([ll, rl])
            ref = np.concatenate([ref, ref2])
        # the same oracle on one thread, on the |k|,|l| <= 4 block
        lo1 = np.array([(k, l) for k in range(-4, 5) for l in range(-4, 5)])
        oracle.threads(1)
        tc = time.perf_counter()
        oracle.cfs_points(clip.xy, clip.off, T, lo1[:, 0], lo1[:, 1])
        t_one = time.perf_counter() - tc
        oracle.threads(cores)
        cpu = {
            "value": V * kk.size / t_pts,
            "unit": "pairs/s",
            "cores": cores,
            "kind": "oracle",
            "sample": (f"same clip, {kk.size} coefficients (the |k|,|l|<=8 block, 400 points "
                       "on the strips 1<=min(|k|,|l|)<=16 and uniform random (k,l)), "
                       f"{t_pts:.1f} s of FP64 edge-form evaluation on {cores} host threads"),
            "single_thread_value": V * lo1.shape[0] / t_one,
            "single_thread_sample": f"same clip, the {lo1.shape[0]} coefficients |k|,|l|<=4",
            "host": host_cpu(),
        }
    f00 = abs(oracle.cfs_points(clip.xy, clip.off, T, [0], [0])[0])
    errs = {}
    for prec, leg in legs.items():
        errs[prec] = float(np.max(np.abs(leg["F"][kk + K, ll + L] - ref)) / f00)
        log(f"{prec}: max err / |F00| over {kk.size} oracle points = {errs[prec]:.3e}")

    main_leg = legs["bf16"]
    ms = main_leg["ms"]
    c_avg = kavg(main_leg["prof"], "contract")
    flops = 3 * 8 * (K + 1) * (L + 1) * V  # three split products, real-trig GEMM
    achieved = flops / (c_avg * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": pairs / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": (f"precision-clip: one layout clip of {V} corners ({clip.n_loops} "
                         f"polygons), T={T}, |k|,|l|<={K} ({2 * K + 1}x{2 * L + 1} complex64 "
                         "coefficients), split-bf16 contraction, FP32 accumulation"),
            "V": V, "T": T, "K": K, "L": L, "precision": "split-bf16",
        },
        "err_rel_f00": errs.get("bf16"),
        "roofline": {
            "bound": "mfma",
            "kernel": "k_contract_split_pipe<bf16> (64x64 frequencies per wave, one wave per SIMD)",
            "achieved": achieved,
            "peak": PEAK_TFLOPS["bf16"],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS["bf16"],
            "traffic": traffic_for("precision-clip/bf16"),
            "kernel_ms": c_avg,
            "flops_per_launch": flops,
        },
        "cpu_baseline": cpu,
        # per-kind kernel times from separate steps with events on every launch
        # (the side-stream figure spans the histograms, guard region and axis DFTs)
        "kernels_ms": main_leg["breakdown"],
        # the streaming steps against the 8 TB/s HBM peak: the pre-pass reads
        # x, y, s (9 B per corner) and writes 16-byte records; the epilogue
        # reads the four FP32 quadrant partials of every split over the
        # computed K x L block and writes the complex64 grid
        "streaming_GBps": streaming_gbps(P, V, T, K, L, main_leg["breakdown"]),
        # 10 further steps timed one by one with events (the paper's protocol
        # of repeated runs): mean +- 95% CI, median
        "step_ms_stats": main_leg["stats"],
        # host canonicalisation of the clip's loops (validation, signs, edge
        # maps), not part of the step
        "canonicalize_host_ms": canon_ms,
        "area_exact": main_leg["area"],
    }
    for prec in ("fp32", "fp16"):
        if prec in legs:
            leg = legs[prec]
            cavg = kavg(leg["prof"], "contract")
            fl = (1 if prec == "fp32" else 3) * 8 * (K + 1) * (L + 1) * V
            out[f"{prec}_form"] = {
                "value": pairs / (leg["ms"] * 1e-3),
                "ms_per_step": leg["ms"],
                "err_rel_f00": errs[prec],
                "contract_ms": cavg,
                "contract_tflops": fl / (cavg * 1e-3) / 1e12,
                "contract_frac": fl / (cavg * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
            }
    if "fp32" in legs:
        out["speedup_vs_fp32"] = legs["fp32"]["ms"] / ms
    if args.quick:
        print(json.dumps(out))
        return 0

    # ------------------------------------------------- lattice (FFT) form, C3
    # The same coefficients from the FP64 lattice form: reported as a separate
    # leg (a different algorithm, not the metric's MFMA contraction), and used
    # as the full-grid reference of the contraction forms.
    Ff = torch.empty_like(F)
    msf, proff = timed(lambda: P.forward_fft(xd, yd, sd, T, K, L, out=Ff), args.steps,
                       args.warmup, h, kinds=("fft",))
    Ff_np = Ff.cpu().numpy().astype(np.complex128)
    ef = float(np.max(np.abs(Ff_np[kk + K, ll + L] - ref)) / f00)
    lattice = {
        "precision_clip": {"value": pairs / (msf * 1e-3), "ms_per_step": msf,
                           "err_rel_f00": ef, "kernels_ms": kavg(proff, "fft")},
    }
    for prec, leg in legs.items():
        out.setdefault("err_full_grid_vs_lattice", {})[prec] = float(
            np.max(np.abs(leg["F"] - Ff_np)) / f00)
    log(f"lattice form: {msf:.3f} ms/step  {pairs / msf * 1e3:.4g} pairs/s  err {ef:.2e}; "
        f"full-grid error of the contraction forms against it: "
        f"{out['err_full_grid_vs_lattice']}")
    del legs

    # ------------------------------------------------------------------ C2
    forms = {}
    T2, K2 = 4096, 255
    c2 = synth.clip(2, T2, K2, n_polygons=2000)
    x2, y2, s2, _, _ = P.loops_to_corners(c2.xy, c2.off)
    x2d, y2d, s2d = (torch.as_tensor(a).to(dev) for a in (x2, y2, s2))
    V2 = int(x2.size)
    p2 = V2 * (2 * K2 + 1) ** 2
    kk2, ll2 = np.meshgrid(np.arange(-6, 7), np.arange(-6, 7), indexing="ij")
    kk2 = np.concatenate([kk2.ravel(), rng.integers(-K2, K2 + 1, 400)])
    ll2 = np.concatenate([ll2.ravel(), rng.integers(-K2, K2 + 1, 400)])
    ref2 = oracle.cfs_points(c2.xy, c2.off, T2, kk2, ll2)
    f002 = abs(oracle.cfs_points(c2.xy, c2.off, T2, [0], [0])[0])
    lay = {"workload": f"layout clip: {V2} corners (2000 polygons), T={T2}, |k|,|l|<={K2}"}
    for prec in ("fp32", "bf16"):
        F2 = torch.empty((2 * K2 + 1, 2 * K2 + 1), dtype=torch.complex64, device=dev)
        ms2, prof2 = timed(lambda: P.forward(x2d, y2d, s2d, T2, K2, K2, precision=prec, out=F2),
                           args.steps, args.warmup, h)
        e2 = float(np.max(np.abs(F2.cpu().numpy()[kk2 + K2, ll2 + K2] - ref2)) / f002)
        lay[prec] = {"value": p2 / (ms2 * 1e-3), "ms_per_step": ms2, "err_rel_f00": e2,
                     "contract_ms": kavg(prof2, "contract")}
        log(f"layout clip {prec}: {ms2:.3f} ms  {p2 / ms2 * 1e3:.4g} pairs/s  err {e2:.2e}")
    forms["layout_clip"] = lay
    F2f = torch.empty((2 * K2 + 1, 2 * K2 + 1), dtype=torch.complex64, device=dev)
    ms2f, _ = timed(lambda: P.forward_fft(x2d, y2d, s2d, T2, K2, K2, out=F2f), args.steps,
                    args.warmup, h, kinds=("fft",))
    e2f = float(np.max(np.abs(F2f.cpu().numpy()[kk2 + K2, ll2 + K2] - ref2)) / f002)
    lattice["layout_clip"] = {"value": p2 / (ms2f * 1e-3), "ms_per_step": ms2f, "err_rel_f00": e2f}
    log(f"layout clip lattice form: {ms2f:.3f} ms  {p2 / ms2f * 1e3:.4g} pairs/s  err {e2f:.2e}")
    forms["lattice_form"] = lattice

    # ------------------------------------------ disjoint (low-fill) variants
    # The same generators with every polygon confined to its own cell of a
    # jittered grid (fill factor well below one, as in a real layer): the
    # error relative to |F[0,0]| is hardest to keep there.
    dis = {}
    for name, seed, Td, Kd, kw in (("layout_clip_disjoint", 22, 4096, 255, {"n_polygons": 2000}),
                                   ("precision_clip_disjoint", 33, 8192, 511,
                                    {"min_vertices": 200_000})):
        cd = synth.clip(seed, Td, Kd, disjoint=True, **kw)
        xdis, ydis, sdis, _, _ = P.loops_to_corners(cd.xy, cd.off)
        xdd, ydd, sdd = (torch.as_tensor(a).to(dev) for a in (xdis, ydis, sdis))
        kkd, lld = np.meshgrid(np.arange(-8, 9), np.arange(-8, 9), indexing="ij")
        kkd = np.concatenate([kkd.ravel(), rng.integers(-Kd, Kd + 1, 300)])
        lld = np.concatenate([lld.ravel(), rng.integers(-Kd, Kd + 1, 300)])
        refd = oracle.cfs_points(cd.xy, cd.off, Td, kkd, lld)
        f00d = abs(oracle.cfs_points(cd.xy, cd.off, Td, [0], [0])[0])
        pd = int(xdis.size) * (2 * Kd + 1) ** 2
        leg = {"workload": (f"{xdis.size} corners ({cd.n_loops} polygons in disjoint cells), "
                            f"T={Td}, |k|,|l|<={Kd}"),
               "fill": f00d * Td / Td ** 2}
        Fd = torch.empty((2 * Kd + 1, 2 * Kd + 1), dtype=torch.complex64, device=dev)
        # full-grid reference: the FP64 lattice form (itself checked against
        # the oracle on the sample)
        Fl, _ = P.forward_fft(xdd, ydd, sdd, Td, Kd, Kd)
        ref_grid = Fl.cpu().numpy().astype(np.complex128)
        leg["lattice_err_rel_f00"] = float(np.max(np.abs(ref_grid[kkd + Kd, lld + Kd] - refd)) / f00d)
        for prec in ("bf16", "fp16", "fp32"):
            msd, _ = timed(lambda: P.forward(xdd, ydd, sdd, Td, Kd, Kd, precision=prec, out=Fd),
                           args.steps, args.warmup, h, kinds=None)
            Fh = Fd.cpu().numpy().astype(np.complex128)
            ed = float(np.max(np.abs(Fh[kkd + Kd, lld + Kd] - refd)) / f00d)
            eg = np.abs(Fh - ref_grid) / f00d
            gi, gj = np.unravel_index(int(np.argmax(eg)), eg.shape)
            leg[prec] = {"value": pd / (msd * 1e-3), "ms_per_step": msd, "err_rel_f00": ed,
                         "err_rel_f00_full_grid": float(eg.max()),
                         "worst_kl": [int(gi - Kd), int(gj - Kd)]}
            log(f"{name} {prec}: {msd:.3f} ms  {pd / msd * 1e3:.4g} pairs/s  err {ed:.2e} sampled, "
                f"{eg.max():.2e} full grid at (k,l)=({gi - Kd},{gj - Kd}) (fill {leg['fill']:.3f})")
        dis[name] = leg
    forms["disjoint"] = dis

    # ------------------------------------------------- pruned Haar transform
    # The PCHT of the same layout clip over its 4096 tile, all 12 wavelet
    # levels (a 4096 x 4096 pyramid of int64 sums and float64 coefficients).
    # Checked bit for bit against the oracle; the oracle's single-threaded
    # time on the whole clip is reported beside it.
    Jh = 12
    off2d = torch.as_tensor(c2.off).to(dev)
    Uh = torch.empty((1 << Jh, 1 << Jh), dtype=torch.int64, device=dev)
    Wh = torch.empty((1 << Jh, 1 << Jh), dtype=torch.float64, device=dev)
    msh, profh = timed(lambda: P.haar(x2d, y2d, s2d, off2d, T2, T2, Jh, out_U=Uh, out_W=Wh),
                       args.steps, args.warmup, h, kinds=("prepass", "haar", "epilogue"))
    _, _, sth = P.haar(x2d, y2d, s2d, off2d, T2, T2, Jh, out_U=Uh, out_W=Wh, stats=True)
    cells, pairs_h = (int(v) for v in sth.cpu().numpy())
    tc = time.perf_counter()
    Uo, Wo, nodes_o = oracle.pcht(c2.xy, c2.off, T2, T2, Jh)
    t_or = time.perf_counter() - tc
    exact = bool(np.array_equal(Uh.cpu().numpy(), Uo)) and cells == nodes_o
    exact_w = bool(np.array_equal(Wh.cpu().numpy(), Wo))
    walk_ms = kavg(profh, "haar")
    # 14 integer operations per (cell, horizontal edge): two clamped widths
    # and two clamped heights (six med3, four subtractions) and four
    # multiply-adds; a loop has one horizontal edge per two corners
    ops = 7 * pairs_h
    peak_alu = 256 * 4 * 16 * 2.4e9 / 1e12  # 32-bit integer VALU, T ops/s
    pyr_bytes = (1 << (2 * Jh)) * 8
    forms["pcht"] = {
        "workload": (f"pruned continuous Haar transform of the layout clip ({c2.n_loops} polygons, "
                     f"{V2} corners), tile {T2} x {T2}, J={Jh} (full {1 << Jh} x {1 << Jh} "
                     "pyramid, int64 sums and float64 coefficients)"),
        "ms_per_step": msh, "cells_visited": cells, "cell_corner_pairs": pairs_h,
        "nonzero_coefficients": int(np.count_nonzero(Uo)),
        "bit_exact_vs_oracle": exact, "coefficients_bit_exact": exact_w,
        "kernels_ms": {"clear_and_plan": kavg(profh, "prepass"), "walk": walk_ms,
                       "scale": kavg(profh, "epilogue")},
        "roofline": {"bound": "alu", "kernel": "k_haar_walk",
                     "achieved": ops / (walk_ms * 1e-3) / 1e12 if walk_ms else None,
                     "peak": peak_alu, "unit": "Tops/s",
                     "frac": ops / (walk_ms * 1e-3) / 1e12 / peak_alu if walk_ms else None},
        "pyramid_passes_GBps": {
            "clear": pyr_bytes / (kavg(profh, "prepass") * 1e-3) / 1e9,
            "scale": 2 * pyr_bytes / (kavg(profh, "epilogue") * 1e-3) / 1e9},
        "cpu_oracle": {"seconds": t_or, "cores": 1, "kind": "oracle",
                       "sample": "the whole clip, all levels"},
    }
    log(f"PCHT: {msh:.3f} ms/step (walk {walk_ms:.3f} ms), {cells} cells, exact {exact}/{exact_w}, "
        f"oracle {t_or:.2f} s")

    # ------------------------------------------------------------------ C1
    # One 64-corner polygon, T = 2048, |k|,|l| <= 64: a latency case (a few
    # microseconds of work).  Timed: the call (one launch of the FP64 direct
    # form at this size), the staged MFMA path forced with a tile variant,
    # and a one-clip captured batch graph; the error is over the whole
    # 129 x 129 grid.
    c1, _, _ = synth.clip_c1(1)
    x1, y1, s1, _, _ = P.loops_to_corners(c1.xy, c1.off)
    x1d, y1d, s1d = (torch.as_tensor(a).to(dev) for a in (x1, y1, s1))
    ref1, area1 = oracle.cfs_grid(c1.xy, c1.off, c1.T, c1.K, c1.L)
    f001 = abs(ref1[c1.K, c1.L])
    p1 = int(x1.size) * (2 * c1.K + 1) * (2 * c1.L + 1)
    single = {"workload": (f"single polygon: {x1.size} corners (union of rectangles), "
                           f"T={c1.T}, |k|,|l|<={c1.K}"), "area": int(area1)}
    n1 = max(50, args.steps * 5)
    for prec in ("fp32", "bf16"):
        F1 = torch.empty((2 * c1.K + 1, 2 * c1.L + 1), dtype=torch.complex64, device=dev)
        a1 = torch.empty(1, dtype=torch.int64, device=dev)
        call = lambda: P.forward(x1d, y1d, s1d, c1.T, c1.K, c1.L, precision=prec, out=F1,
                                 area_out=a1)
        ms1, _ = timed(call, n1, 5, h, kinds=None)
        _, pr1 = timed(call, n1, 0, h, kinds=("direct",))
        e1 = float(np.max(np.abs(F1.cpu().numpy().astype(np.complex128) - ref1)) / f001)
        mss, _ = timed(lambda: P.forward(x1d, y1d, s1d, c1.T, c1.K, c1.L, precision=prec,
                                         out=F1, area_out=a1, tile=0), n1, 5, h, kinds=None)
        es = float(np.max(np.abs(F1.cpu().numpy().astype(np.complex128) - ref1)) / f001)
        b1 = P.Batch([(x1d, y1d, s1d, c1.T, c1.K, c1.L)], precision=prec)
        msg, _ = timed(b1.run, n1, 5, h, kinds=None)
        eg = float(np.max(np.abs(b1.F[0].cpu().numpy().astype(np.complex128) - ref1)) / f001)
        single[prec] = {"us_per_call": ms1 * 1e3, "direct_kernel_us": kavg(pr1, "direct") * 1e3,
                        "us_per_call_staged": mss * 1e3, "err_rel_f00_staged": es,
                        "us_per_graph_replay": msg * 1e3,
                        "value": p1 / (ms1 * 1e-3), "err_rel_f00": max(e1, eg),
                        "area_exact": int(a1.item()) == int(area1)
                        and int(b1.area[0].item()) == int(area1)}
        b1.close()
        log(f"single polygon {prec}: {ms1 * 1e3:.1f} us per call (direct kernel "
            f"{kavg(pr1, 'direct') * 1e3:.1f} us), staged {mss * 1e3:.1f} us, "
            f"{msg * 1e3:.1f} us per graph replay, err {max(e1, eg):.2e}")
    forms["single_polygon"] = single

    # ------------------------------------------------------------- general tile
    # Periods that are neither equal nor powers of two, and a finer corner
    # grid: the precision clip on an 8000 x 6000 tile (K = L = 511, same
    # corners and coefficient count as the headline), and the layout clip drawn
    # on half units over a 4000 x 3000 tile (periods 8000 x 6000 grid units).
    # The third: the layout clip on a 4000 x 3000 tile with every polygon
    # shifted by its own random multiple of 1/16 (periods 64000 x 48000 grid
    # units, past the LDS tables: two-level twiddles).  The fourth: the
    # precision clip on an 8000 x 6000 tile, polygons shifted by multiples of
    # 1/8 (periods 64000 x 48000 grid units, the two-level kernel at the
    # headline's size).
    import types

    def shifted(cl, fb):
        Xs = cl.xy.astype(np.int64) << fb
        for i in range(cl.off.size - 1):
            Xs[cl.off[i]:cl.off[i + 1]] += rng.integers(0, 1 << fb, 2)
        cs = types.SimpleNamespace(xy=Xs.astype(np.int32), off=cl.off)
        xs, ys, ss, _, _ = P.loops_to_corners(cs.xy, cs.off)
        return (cs,) + tuple(torch.as_tensor(a).to(dev) for a in (xs, ys, ss))

    c16, x16d, y16d, s16d = shifted(c2, 4)
    c8, x8d, y8d, s8d = shifted(clip, 3)
    gen = {}
    for name, gclip, gx, gy, gs, Ng, Mg, Fb, Kg in (
            ("precision_clip_8000x6000", clip, xd, yd, sd, 8000, 6000, 0, K),
            ("layout_clip_half_units_4000x3000", c2, x2d, y2d, s2d, 4000, 3000, 1, K2),
            ("layout_clip_sixteenth_units_4000x3000", c16, x16d, y16d, s16d, 4000, 3000, 4, K2),
            ("precision_clip_eighth_units_8000x6000", c8, x8d, y8d, s8d, 8000, 6000, 3, K)):
        Vg = int(gx.numel())
        pg = Vg * (2 * Kg + 1) ** 2
        kq = np.concatenate([kk[:289] if Kg >= 8 else kk, rng.integers(-Kg, Kg + 1, 200)])
        lq = np.concatenate([ll[:289] if Kg >= 8 else ll, rng.integers(-Kg, Kg + 1, 200)])
        xyg = gclip.xy.astype(np.float64) / 2 ** Fb
        refg = oracle.cfs_points_general(xyg, gclip.off, Ng, Mg, kq, lq, frac_bits=Fb)
        f00g = abs(oracle.cfs_points_general(xyg, gclip.off, Ng, Mg, [0], [0], frac_bits=Fb)[0])
        entry = {"workload": (f"{Vg} corners, tile {Ng} x {Mg}, corners on a 2^-{Fb} grid "
                              f"(periods {Ng << Fb} x {Mg << Fb} grid units), |k|,|l|<={Kg}")}
        Fgen = torch.empty((2 * Kg + 1, 2 * Kg + 1), dtype=torch.complex64, device=dev)
        for prec in ("fp32", "bf16"):
            msg, profg = timed(lambda: P.forward_general(gx, gy, gs, Ng, Mg, Kg, Kg, frac_bits=Fb,
                                                         precision=prec, out=Fgen),
                               args.steps, args.warmup, h)
            eg = float(np.max(np.abs(Fgen.cpu().numpy()[kq + Kg, lq + Kg] - refg)) / f00g)
            cms = kavg(profg, "contract")
            fl = (3 if prec != "fp32" else 1) * 8 * (Kg + 1) ** 2 * Vg
            entry[prec] = {"value": pg / (msg * 1e-3), "ms_per_step": msg, "err_rel_f00": eg,
                           "contract_ms": cms,
                           "roofline": {"bound": "mfma", "achieved": fl / (cms * 1e-3) / 1e12,
                                        "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                                        "frac": fl / (cms * 1e-3) / 1e12 / PEAK_TFLOPS[prec]}}
            log(f"general tile {name} {prec}: {msg:.3f} ms  {pg / msg * 1e3:.4g} pairs/s  "
                f"err {eg:.2e}  contract {cms:.3f} ms")
        gen[name] = entry
    # Batch of general tiles in one captured graph: 32 clips of 150-600
    # polygons on tiles of random periods (1000..6000 lattice units, grid
    # steps 2^-F with F in 0..4, some past 8192 grid units), K = L = 127.
    gclips, gpairs = [], 0
    grng = np.random.default_rng(77)
    for i in range(32):
        Ngx, Ngy = (int(v) for v in grng.integers(1000, 6001, 2))
        Fq = int(grng.integers(0, 5))
        cg = synth.clip(500 + i, max(Ngx, Ngy), 127, n_polygons=int(grng.integers(150, 601)))
        Xg = cg.xy.astype(np.int64) << Fq
        for j in range(cg.off.size - 1):
            Xg[cg.off[j]:cg.off[j + 1]] += grng.integers(0, 1 << Fq, 2)
        gxg, gyg, gsg, _, _ = P.loops_to_corners(Xg.astype(np.int32), cg.off)
        gclips.append((gxg, gyg, gsg, Ngx, Ngy, 127, 127, Fq))
        gpairs += int(gxg.size) * 255 * 255
    gb = P.GeneralBatch(gclips, precision="bf16")
    msb, _ = timed(gb.run, args.steps, args.warmup, h, kinds=None)
    gb.close()
    gen["batch_32_general_tiles"] = {
        "workload": (f"32 clips, {sum(int(c[0].numel()) for c in gb.corners)} corners, periods "
                     "1000..6000 lattice units on grids of step 2^-F (F in 0..4), K = L = 127, "
                     "one graph replay"),
        "bf16": {"value": gpairs / (msb * 1e-3), "ms_per_step": msb}}
    log(f"general batch of 32 tiles bf16: {msb:.3f} ms per replay  {gpairs / msb * 1e3:.4g} pairs/s")
    forms["general_tile"] = gen

    # ------------------------------------------------------------------ C4
    t0 = time.time()
    bclips = synth.batch_clips(4, n_clips=256)
    bargs = []
    bpairs = 0
    bflops = 0
    for c in bclips:
        bx, by, bs, _, _ = P.loops_to_corners(c.xy, c.off)
        bargs.append((bx, by, bs, c.T, c.K, c.L))
        bpairs += int(bx.size) * (2 * c.K + 1) * (2 * c.L + 1)
        bflops += 3 * 8 * (c.K + 1) * (c.L + 1) * int(bx.size)
    nvb = sum(int(a[0].size) for a in bargs)
    log(f"batch: 256 clips, {nvb} corners, {bpairs:.3e} pairs (generated in "
        f"{time.time() - t0:.1f}s)")
    # tile shape and corners per work item from the library's batch autotuner,
    # timed on these clips
    t0 = time.time()
    batch = P.Batch(bargs, precision="bf16", tune=True)
    t_tune = time.time() - t0
    log(f"batch autotune: {t_tune:.1f}s, choice per K bucket (tile variant, corners per item) "
        f"{batch.choice}")
    msb, profb = timed(batch.run, max(3, args.steps // 4), 1, h, kinds=("batch",))
    # error on the four smallest clips and four random ones, sampled points
    order = np.argsort([int(a[0].size) for a in bargs])
    pick = list(order[:4]) + list(rng.choice(order[4:], 4, replace=False))
    eb = 0.0
    for i in pick:
        c = bclips[i]
        kq, lq = (rng.integers(-c.K, c.K + 1, 64), rng.integers(-c.L, c.L + 1, 64))
        kq = np.concatenate([kq, [1, 1, 2, -1]])
        lq = np.concatenate([lq, [1, -1, 1, 2]])
        rq = oracle.cfs_points(c.xy, c.off, c.T, kq, lq)
        fq = abs(oracle.cfs_points(c.xy, c.off, c.T, [0], [0])[0])
        got = batch.F[i].cpu().numpy()[kq + c.K, lq + c.L]
        eb = max(eb, float(np.max(np.abs(got - rq)) / fq))
    forms["batch"] = {
        "workload": ("256 clips, corners log-uniform in [1k, 200k], (T,K) uniform over "
                     "{(1024,63),(2048,127),(4096,255),(8192,511)}, split-bf16, one graph replay"),
        "clips": 256, "corners": nvb, "pairs": bpairs,
        "value": bpairs / (msb * 1e-3), "ms_per_step": msb,
        "err_rel_f00_max_of_8_clips": eb,
        # algorithmic split-bf16 flops of all clips over the whole graph replay
        # (every kernel of the batch counted in the time)
        "roofline": {"bound": "mfma", "achieved": bflops / (msb * 1e-3) / 1e12,
                     "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                     "frac": bflops / (msb * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"]},
        "autotune": {"seconds": t_tune,
                     "per_kbucket": {f"K<={P.BATCH_KBUCKET_MAX[kb]}" if kb < 4 else "K>511":
                                     {"tile_variant": t, "corners_per_item": ch}
                                     for kb, (t, ch) in batch.choice.items()}},
    }
    log(f"batch: {msb:.3f} ms  {bpairs / msb * 1e3:.4g} pairs/s  err {eb:.2e}")
    batch.close()
    del batch

    # ----------------------------------------- paper-shaped tiles (context)
    # The paper's own regime: 1024 x 1024 tiles (1 nm units) with the full
    # 1023 x 1023 grid (|k|,|l| <= 511) and about 60 corners each (the paper's
    # ~11 shapes per tile are mostly rectangles; this generator's polygons are
    # unions of up to 10 rectangles, so 4 of them give that corner count);
    # 256 tiles in one graph replay.  At ~60 corners a tile is bound by its
    # 8.4 MB output write.  The per-tile time sits beside the paper's CPU figure for
    # its own method variant on other hardware: context, not a target.
    Tp, Kp, ntp = 1024, 511, 256
    ptiles = [synth.clip(7000 + i, Tp, Kp, n_polygons=4) for i in range(ntp)]
    pargs, ppairs = [], 0
    for c in ptiles:
        px, py, ps, _, _ = P.loops_to_corners(c.xy, c.off)
        pargs.append((px, py, ps, Tp, Kp, Kp))
        ppairs += int(px.size) * (2 * Kp + 1) ** 2
    pb = P.Batch(pargs, precision="bf16", tune=True)  # the autotuner picks for these tiles
    msp, _ = timed(pb.run, max(3, args.steps // 4), 1, h, kinds=None)
    ep = 0.0
    for i in (0, 1):
        refp, _ = oracle.cfs_grid(ptiles[i].xy, ptiles[i].off, Tp, Kp, Kp)
        got = pb.F[i].cpu().numpy().astype(np.complex128)
        ep = max(ep, float(np.max(np.abs(got - refp)) / abs(refp[Kp, Kp])))
    nvp = sum(int(a[0].size) for a in pargs)
    forms["paper_shaped_tiles"] = {
        "workload": (f"{ntp} tiles of 1024 x 1024 (4 polygons, {nvp / ntp:.0f} corners on "
                     "average), full 1023 x 1023 grid, split-bf16, one graph replay"),
        "us_per_tile": msp * 1e3 / ntp, "ms_per_step": msp,
        "value": ppairs / (msp * 1e-3), "unit": "pairs/s",
        "output_GBps": ntp * (2 * Kp + 1) ** 2 * 8 / (msp * 1e-3) / 1e9,
        "err_rel_f00_full_grid_2_tiles": ep,
        "autotune": {"tile_variant": pb.choice[3][0], "corners_per_item": pb.choice[3][1]},
        "paper_cpu_us_per_tile": 15648.0,
    }
    log(f"paper-shaped tiles: {msp * 1e3 / ntp:.2f} us per tile "
        f"({forms['paper_shaped_tiles']['output_GBps']:.0f} GB/s of output), err {ep:.2e}, "
        f"choice {pb.choice[3]}")
    pb.close()
    del pb

    # ------------------------------------------------------------------ C5
    T5, K5 = 4096, 255
    r5 = 0.35 * K5
    rb = int(np.floor(r5))
    c5 = synth.clip(5, T5, K5, min_vertices=100_000)
    # the optimisation loop's offsets lie on the lattice by construction: no
    # per-call host comparison (which would wait for the device every step)
    geom = P.Geometry(c5.xy, c5.off, T5, K5, check_offsets=False)
    kk5, ll5 = np.meshgrid(np.arange(-K5, K5 + 1), np.arange(-K5, K5 + 1), indexing="ij")
    Hp = ((kk5 ** 2 + ll5 ** 2) <= r5 * r5).astype(np.float32)
    Hd = torch.as_tensor(Hp).to(dev)
    # target: pupil-filtered spectrum of a second clip.  For the gradient check
    # it comes from the oracle (an input to both sides); for timing alone the
    # GPU forward provides it.
    c6 = synth.clip(6, T5, K5, min_vertices=100_000)
    kb5, lb5 = np.nonzero(Hp)
    if args.check_adjoint:
        Gt_np = np.zeros(Hp.shape, np.complex128)
        Gt_np[kb5, lb5] = oracle.cfs_points(c6.xy, c6.off, T5, kb5 - K5, lb5 - K5)
        Gt = torch.as_tensor(Gt_np.astype(np.complex64)).to(dev)
    else:
        x6, y6, s6, _, _ = P.loops_to_corners(c6.xy, c6.off)
        Gt, _ = P.forward(x6, y6, s6, T5, K5, K5, precision="fp32")
        Gt = Hd * Gt
    off = torch.zeros(geom.n_edges, dtype=torch.float32, device=dev, requires_grad=True)

    def step5():
        off.grad = None
        # low-pass forward and its adjoint: only the pupil's band and disc;
        # the loss and its cotangent in one kernel
        Fv = P.FCFSFunction.apply(off, geom, "bf16", (rb, rb), r5)
        loss = P.PupilLoss.apply(Fv, Gt, r5)
        loss.backward()

    def step5_torch_loss():
        off.grad = None
        Fv = P.FCFSFunction.apply(off, geom, "bf16", (rb, rb), r5)
        loss = ((Hd * Fv - Gt).abs() ** 2).sum()
        loss.backward()

    ms5t, _ = timed(step5_torch_loss, max(3, args.steps // 4), 1, h)
    ms5, prof5 = timed(step5, max(3, args.steps // 4), 1, h,
                       kinds=("prepass", "contract", "epilogue", "adjoint", "adjoint_gemm"))
    # the same step as one library call (fcfs_pupil_step): identical launches
    # without the autograd engine between them; its gradient is compared with
    # the autograd step's bit for bit
    off0 = off.detach().clone()
    ms5s, _ = timed(lambda: P.pupil_step(geom, off0, Gt, radius=r5, band=(rb, rb)),
                    max(3, args.steps // 4), 1, h, kinds=None)
    step5()
    _, g_one = P.pupil_step(geom, off0, Gt, radius=r5, band=(rb, rb))
    one_call_same = bool(torch.equal(g_one, off.grad))
    # and captured once into a graph, replayed per step (new offsets copied in)
    plan5 = P.PupilStep(geom, Gt, radius=r5, band=(rb, rb))
    ms5g, _ = timed(lambda: plan5.run(off0), max(3, args.steps // 4), 1, h, kinds=None)
    _, g_graph = plan5.run(off0)
    graph_same = bool(torch.equal(g_graph, off.grad))
    plan5.close()
    V5 = int(geom.base_x.numel())
    adj = {
        "workload": (f"adjoint: {V5} corners, T={T5}, |k|,|l|<={K5}, loss sum |H F - G|^2 with a "
                     f"circular pupil of radius {r5:.2f}; low-pass forward + backward over the "
                     "pupil, split-bf16; the loss and its cotangent in one kernel (the step with "
                     "the loss in torch ops is reported beside it)"),
        "ms_per_step": ms5,
        "ms_per_step_loss_in_torch_ops": ms5t,
        "ms_per_step_one_call": ms5s,
        "one_call_gradient_equals_autograd": one_call_same,
        "ms_per_step_graph_replay": ms5g,
        "graph_gradient_equals_autograd": graph_same,
        "forward_ms": sum(kavg(prof5, k) or 0.0 for k in ("prepass", "contract", "epilogue")),
        "adjoint_ms": kavg(prof5, "adjoint"),
        "adjoint_gemm_ms": kavg(prof5, "adjoint_gemm"),
        "value": V5 * (2 * K5 + 1) ** 2 / (ms5 * 1e-3),
    }
    # adjoint GEMM work inside the pupil band (three split products of the
    # 2 kmax x 4 lmax folded cotangent per corner): over the main-term kernel
    # alone (events around its launch), and over all adjoint kernels
    aflops = 3 * 2 * (2 * rb) * (4 * rb) * V5
    if adj["adjoint_gemm_ms"]:
        tf = aflops / (adj["adjoint_gemm_ms"] * 1e-3) / 1e12
        adj["roofline"] = {"bound": "mfma",
                           "kernel": "k_adj_gemm_regb<bf16> (main term, W resident in registers)",
                           "achieved": tf, "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                           "frac": tf / PEAK_TFLOPS["bf16"], "flops_per_launch": aflops}
    if adj["adjoint_ms"]:
        tf = aflops / (adj["adjoint_ms"] * 1e-3) / 1e12
        adj["roofline_all_adjoint_kernels"] = {"achieved": tf, "unit": "TFLOP/s",
                                               "frac": tf / PEAK_TFLOPS["bf16"]}
    if args.check_adjoint:
        # gradient check on sampled edges against the FP64 oracle
        Fo = np.zeros(Hp.shape, np.complex128)
        Fo[kb5, lb5] = oracle.cfs_points(c5.xy, c5.off, T5, kb5 - K5, lb5 - K5)
        Go = 2 * Hp * (Hp * Fo - Gt_np.astype(np.complex64).astype(np.complex128))
        edges = rng.choice(geom.n_edges, 128, replace=False)
        want = oracle.edge_grad(c5.xy, c5.off, T5, K5, K5, Go, edges=edges)
        step5()
        got = off.grad.detach().cpu().numpy().astype(np.float64)[edges]
        adj["grad_err_rel_max"] = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    forms["adjoint"] = adj
    log(f"adjoint: main-term kernel {adj['adjoint_gemm_ms']:.4f} ms "
        f"({adj.get('roofline', {}).get('frac', 0.0):.3f} of bf16 peak), all adjoint kernels "
        f"{adj['adjoint_ms']:.4f} ms")
    log(f"adjoint: {ms5:.3f} ms per forward+backward (loss in torch ops: {ms5t:.3f} ms; "
        f"one library call {ms5s:.3f} ms, same gradient: {one_call_same}; captured step "
        f"{ms5g:.3f} ms per replay, same gradient: {graph_same})")
    out["forms"] = forms
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
