#!/usr/bin/env python3
"""Throughput of the LLOID filtering path on one MI355X.

Workload (the multi-rate configuration the metric is quoted on): one SVD
bank of 1024 synthetic chirp templates (durations 0.5-32 s) in three time
slices at 2048/512/128 Hz with 200/150/100 basis filters, two detectors of
1024 s of white Gaussian noise with 20 injections (SNR 6-30), 1 s trigger
windows, threshold 4.  One step filters both detectors from strain already
resident in HBM to triggers in pinned host memory, through the C ABI.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--compute f16|bf16|f32]

Prints one JSON line: whole-job template-samples of SNR per second, the
roofline of the dominant kernel (device time from HIP events on the
library's stream over the timed steps), the plain FP32 and the BF16 paths
beside it, the SNR-series output mode (HBM-bound), the same path with every
trigger's xi2 signal-consistency value (bank autocorrelations over 2K + 1
lags), the latency of the 64-template single-rate block, the conditioning of
one detector's block (PSD, whitening, gating), the coincidence of the two
detectors' triggers, the batched form (64 uneven banks) and the serving form
(128 banks streamed in 1 s strides: p50/p99 stride latency at 16x real time
and at saturation), and the FP64 oracle timed on the host cores (one
single-threaded process per core over disjoint ranges) on a bounded sample.
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

METRIC = "template-samples of SNR/sec (1 GPU) at stated SNR error; p99 stride latency"
PEAK_TFLOPS = {"f16": 2516.6, "bf16": 2516.6, "f32": 157.3}   # dense MFMA, MI355X
PEAK_HBM_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_2410_16416_amd", "csrc", "lloid_kernels.hip")
TILE_CACHE = os.path.join(ROOT, "paper_2410_16416_amd", "tiles_gfx950.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stage_work(bank, seconds: float, compute: str):
    """Algorithmic work per lloid_filter call (one detector), per stage.

    FIR: 2 L_s N_s r_s flops per second of data; mixing: 2 (2F) L_s r_s
    (the method's order: mix at the slice rate).  Interpolation moves the
    low-rate orthogonal SNR (read once, in the low-rate buffer type: FP32 for
    f32 and bf16 operands) to the full-rate operand (written once)."""
    esz = 4 if compute == "f32" else 2
    lsz = 2 if compute == "f16" else 4
    fir = sum(2.0 * s.n_basis * s.n_taps * s.rate for s in bank.slices) * seconds
    mix = sum(2.0 * 2 * bank.n_templates * s.n_basis * s.rate for s in bank.slices) * seconds
    interp = sum((s.n_basis * s.rate * lsz + s.n_basis * bank.f0 * esz)
                 for s in bank.slices if s.rate != bank.f0) * seconds
    decim = sum(4.0 * bank.f0 / 2 ** k * 1.5 for k in range(1, 5)) * seconds
    return {"fir": ("mfma", fir), "mix": ("mfma", mix), "interp": ("hbm", interp), "decimate": ("hbm", decim)}


def roofline_entry(kind, work, ms_per_launch, compute, traffic=None):
    if kind == "mfma":
        achieved = work / (ms_per_launch / 1e3) / 1e12
        peak = PEAK_TFLOPS[compute]
        return {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic}
    achieved = work / (ms_per_launch / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic}


def load_traffic(stage: str, compute: str):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(PROFILES, f"traffic_{stage}_multirate_c1_{compute}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sha") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline_1thread(wl, sample_s: float):
    """The oracle on one BLAS thread in this process (the paper's single-CPU-core
    framing): detector 0, outputs on [32 s, 32 s + sample_s)."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:
        return None
    with threadpool_limits(limits=1):
        r = _oracle_range(wl.bank, wl.strains[0], 32.0, 32.0 + sample_s, 1.0)
    return {"value": round(r["samples"] / r["wall"], 1), "unit": "template-samples/s", "cores": 1,
            "kind": "oracle",
            "sample": f"detector 0, outputs on [32 s, {32 + sample_s:g} s) of the same workload (all "
                      f"{wl.bank.n_templates} templates, 32 s history), FP64 NumPy/SciPy multi-rate form plus "
                      f"window peaks and triggers; wall {r['wall']:.2f} s on 1 BLAS thread"}


def _oracle_range(bank, x, s_lo: float, s_hi: float, piece_s: float):
    """Oracle outputs and triggers of x on [s_lo, s_hi) seconds in pieces of
    piece_s seconds (bounded memory), timed."""
    import oracle
    f0 = bank.f0
    t0 = time.perf_counter()
    n_trig = 0
    a = int(s_lo * f0)
    end = int(s_hi * f0)
    # each piece starts its strain 34 s (the longest filter plus the resampler
    # halos) before its outputs, at a multiple of 2^7 samples: the multi-rate
    # form is shift-equivariant by such multiples, so the outputs are those of
    # the whole block
    hist = 34 * f0
    while a < end:
        b = min(end, a + int(piece_s * f0))
        o = max(0, (a - hist) // 128 * 128)
        z = oracle.lloid_snr(bank, x[o: b + 4 * f0], a - o, b - o)
        n_trig += len(oracle.triggers(z, a, f0, 1, 1, 4.0))
        a = b
    return {"samples": bank.n_templates * (end - int(s_lo * f0)), "wall": time.perf_counter() - t0,
            "triggers": n_trig}


def _cpu_worker(bank, x, s_lo, s_hi):
    """One single-threaded oracle process (spawned: BLAS threads limited before
    numpy is imported)."""
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        return _oracle_range(bank, x, s_lo, s_hi, 8.0)


def cpu_baseline(wl, seconds_per_worker: float, workers: int):
    """The FP64 oracle on the host cores: `workers` single-threaded processes,
    each computing detector 0's outputs on its own disjoint range of
    seconds_per_worker seconds from 32 s on (the oracle's sub-range
    evaluation, each range with the history it needs); the value is all
    ranges' template-samples over the wall time from the first start to the
    last end.  Run before the GPU is initialised."""
    import concurrent.futures as cf
    import multiprocessing as mp
    f0 = wl.bank.f0
    total_s = wl.n_samples / f0
    workers = max(1, min(workers, int((total_s - 32) // seconds_per_worker)))
    ranges = [(32 + k * seconds_per_worker, 32 + (k + 1) * seconds_per_worker) for k in range(workers)]
    x = wl.strains[0][: int(ranges[-1][1] * f0) + 4 * f0]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        # start every worker (imports done) before the clock starts
        list(ex.map(_cpu_warm, range(workers)))
        t0 = time.perf_counter()
        res = list(ex.map(_cpu_worker, [wl.bank] * workers, [x] * workers, [r[0] for r in ranges],
                          [r[1] for r in ranges]))
        wall = time.perf_counter() - t0
    samples = sum(r["samples"] for r in res)
    return {"value": round(samples / wall, 1), "unit": "template-samples/s", "cores": workers, "kind": "oracle",
            "sample": f"detector 0, outputs on [32 s, {ranges[-1][1]:g} s) of the same workload (all "
                      f"{wl.bank.n_templates} templates) split into {workers} disjoint ranges of "
                      f"{seconds_per_worker:g} s, one single-threaded process each with its own history; "
                      f"FP64 NumPy/SciPy multi-rate form plus window peaks and triggers; wall {wall:.2f} s "
                      f"({os.cpu_count()} host cores visible)",
            "triggers": int(sum(r["triggers"] for r in res))}


def _cpu_warm(_):
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import numpy  # noqa: F401
    import scipy.signal  # noqa: F401
    import oracle  # noqa: F401
    return 0


def run_path(lloid, ctx, wl, xs, compute, steps, warmup, tbufs, args):
    import torch
    bank = lloid.bank_from_svd(ctx, wl.bank, compute)
    try:
        if compute != "f32" or args.compute == "f32":
            tiles = pick_tiles(lloid, ctx, [bank], args)
        else:   # the plain FP32 reference path keeps the default tiles
            lloid.lloid_ctx_set_tiles(ctx, 0, 0)
            tiles = {"fir_variant": 0, "mix_variant": 0, "source": "defaults"}
        def step():
            n = 0
            for det, x in enumerate(xs):
                r = lloid.lloid_filter(bank, det, x, window=(1, 1), threshold=4.0, triggers_out=tbufs[det])
                n += r.n_triggers
            return n

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        lloid.lloid_ctx_profile(ctx, True)
        lloid.lloid_ctx_stage_times(ctx, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_trig = 0
        for _ in range(steps):
            n_trig = step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stages = lloid.lloid_ctx_stage_times(ctx, reset=True)
        lloid.lloid_ctx_profile(ctx, False)
    finally:
        lloid.lloid_bank_destroy(bank)
    return wall, n_trig, stages, tiles


def pick_tiles(lloid, ctx, handles, args):
    """Tile variants for these banks: the recorded autotuning choice, or a new
    timing over args.tune_seconds of synthetic strain (recorded in the cache)."""
    if args.tune_seconds == 0:
        fv, mv = lloid.lloid_ctx_get_tiles(ctx)
        return {"fir_variant": fv, "mix_variant": mv, "source": "context (no autotuning)"}
    seconds = args.tune_seconds if args.tune_seconds > 0 else args.block_seconds
    (fv, mv), res = lloid.lloid_autotune(ctx, handles, seconds, args.tile_cache)
    return {"fir_variant": fv, "mix_variant": mv, "source": "timed" if len(res) else "cache",
            "cache": os.path.relpath(args.tile_cache, ROOT) if args.tile_cache.startswith(ROOT) else args.tile_cache}


def batched_work(banks, seconds):
    fir = sum(2.0 * s.n_basis * s.n_taps * s.rate for b in banks for s in b.slices) * seconds
    mix = sum(2.0 * 2 * b.n_templates * s.n_basis * s.rate for b in banks for s in b.slices) * seconds
    return fir, mix


def measure_batched(lloid, ctx, banks, xs, compute, steps, warmup, seconds, args, tiles_from_cache=True):
    """One step filters both detectors' strain (device) with every bank
    (lloid_filter_batch, one launch per stage per chunk); returns the step's
    throughput, wall time and algorithmic MFMA fraction."""
    import torch
    hs = [lloid.bank_from_svd(ctx, b, compute) for b in banks]
    try:
        if tiles_from_cache:
            tiles = pick_tiles(lloid, ctx, hs, args)
        else:   # the plain FP32 reference path keeps the default tiles
            lloid.lloid_ctx_set_tiles(ctx, 0, 0)
            tiles = {"fir_variant": 0, "mix_variant": 0, "source": "defaults"}
        cap = sum(b.n_templates for b in banks) * seconds
        tbuf = torch.empty(cap * lloid.TRIGGER_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)

        def step():
            n = 0
            for d, x in enumerate(xs):
                n += lloid.lloid_filter_batch(hs, d, x, window=(1, 1), triggers_out=tbuf).n_triggers
            return n
        for _ in range(max(warmup, 1)):
            step()
        torch.cuda.synchronize()
        lloid.lloid_ctx_profile(ctx, True)
        lloid.lloid_ctx_stage_times(ctx, reset=True)
        t = time.perf_counter()
        for _ in range(steps):
            ntr = step()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / steps
        stages = lloid.lloid_ctx_stage_times(ctx, reset=True)
        lloid.lloid_ctx_profile(ctx, False)
    finally:
        for h in hs:
            lloid.lloid_bank_destroy(h)
    f0 = banks[0].f0
    samples = sum(b.n_templates for b in banks) * seconds * f0 * len(xs)
    fir, mix = batched_work(banks, seconds * len(xs))
    return {"value": round(samples / wall, 1), "ms_per_step": round(wall * 1e3, 2), "steps": steps,
            "triggers_per_step": int(ntr),
            "algorithmic_tflop_per_step": round((fir + mix) / 1e12, 2),
            "algorithmic_tflops": round((fir + mix) / wall / 1e12, 1),
            "mfma_frac_of_peak": round((fir + mix) / wall / 1e12 / PEAK_TFLOPS[compute], 4),
            "stage_ms_per_step": {k: round(v[0] / steps, 3) for k, v in stages.items()},
            "tiles": tiles}


def bench_batched(args):
    """64 uneven banks (F 200-2000, 1-4 slices, filters 0.5-64 s), 2 detectors x
    512 s; one step filters both detectors with every bank, one launch per
    stage per chunk (lloid_filter_batch)."""
    import numpy as np
    import torch
    from workloads import configs
    from paper_2410_16416_amd import lloid
    nb = args.banks or 64
    seconds = args.seconds if args.seconds != 1024 else 512
    args.block_seconds = seconds
    log(f"[bench] batched: generating {nb} banks")
    t0 = time.perf_counter()
    banks = configs.batched_c3_banks(nb)
    log(f"[bench] banks ready in {time.perf_counter() - t0:.1f} s")
    f0 = 2048
    xs = [torch.from_numpy(np.random.default_rng(configs.seed(3, d)).standard_normal(seconds * f0)).to("cuda")
          for d in range(2)]
    torch.cuda.init()
    ctx = lloid.lloid_ctx_create(0)
    out = {}
    for compute in [args.compute] + (["f32"] if args.f32_steps and args.compute != "f32" else []):
        main_ = compute == args.compute
        out[compute] = measure_batched(lloid, ctx, banks, xs, compute, args.steps if main_ else args.f32_steps,
                                       args.warmup if main_ else 1, seconds, args, tiles_from_cache=main_)
        log(f"[bench] batched {compute}: {out[compute]}")
    lloid.lloid_ctx_destroy(ctx)
    main_ = out[args.compute]
    return {"metric": METRIC, "value": main_["value"], "unit": "template-samples/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.compute,
            "data": "synthetic (seeded white Gaussian noise; uneven bank shapes with seeded random orthonormal bases)",
            "config": {"workload": f"batched_c3: {nb} uneven SVD banks (F U[200,2000], 1-4 slices at 2048 Hz "
                                   f"and lower, filters 0.5-64 s), 2 detectors x {seconds} s, one launch per stage",
                       "banks": nb, "templates": sum(b.n_templates for b in banks), "detectors": 2,
                       "seconds": seconds, "f0": f0},
            "paths": out}


def measure_serving(lloid, ctx, banks, hs, compute, rate, n_str, xs, use_graph=False, warm=4):
    """Push n_str 1 s strides of 2 detectors (after `warm` untimed ones) at
    `rate` x real time (0: as fast as the stream takes them) into a stream
    holding every bank of hs; latency of each stride from its push to its
    triggers being visible to the host (the library's clock), throughput over
    the wall time of the timed strides."""
    import numpy as np
    f0 = banks[0].f0
    total = xs[0].shape[0] // f0
    s = lloid.lloid_stream_create(ctx, f0, compute, n_detectors=2, min_rate_hz=128, window=(1, 1),
                                  max_filter_s=66.0, max_windows_per_tick=2, use_graph=use_graph)
    try:
        for h in hs:
            lloid.lloid_stream_admit(s, h)
        n_trig = 0
        t_start = None
        for i in range(n_str + warm):
            if i == warm:
                lloid.lloid_stream_poll(s, wait_ms=-1)      # the warm-up strides are done
                lloid.lloid_stream_stats_reset(s)
                t_start = time.perf_counter()
            if t_start is not None and rate > 0:
                due = t_start + (i - warm) / rate
                while time.perf_counter() < due:
                    pass
            j = i % total   # strain cycles through the generated seconds
            for d in range(2):
                lloid.lloid_stream_push(s, d, i * f0, xs[d][j * f0:(j + 1) * f0])
            if i >= warm:
                n_trig += lloid.lloid_stream_poll(s).shape[0]
        n_trig += lloid.lloid_stream_poll(s, wait_ms=-1).shape[0]
        wall = time.perf_counter() - t_start
        st = lloid.lloid_stream_stats_get(s)
    finally:
        lloid.lloid_stream_destroy(s)
    samples = sum(b.n_templates for b in banks) * n_str * f0 * 2
    fir, mix = batched_work(banks, n_str * 2)
    return {"value": round(samples / wall, 1), "wall_s": round(wall, 3), "strides": n_str,
            "rate_x_real_time": rate if rate > 0 else "saturation",
            "p50_stride_latency_ms": round(st.latency_p50_ms, 3),
            "p99_stride_latency_ms": round(st.latency_p99_ms, 3),
            "max_stride_latency_ms": round(st.latency_max_ms, 3),
            "ms_per_stride": round(wall / n_str * 1e3, 3),
            "mfma_frac_of_peak": round((fir + mix) / wall / 1e12 / PEAK_TFLOPS[compute], 4),
            "kept_up": bool(rate <= 0 or wall <= n_str / rate * 1.05), "triggers": int(n_trig),
            "hip_graph": bool(use_graph), "graph_captures": int(st.graph_captures),
            "graph_replays": int(st.graph_replays)}


def serving_inputs(seconds: int = 64):
    import numpy as np
    from workloads import configs
    return [np.random.default_rng(configs.seed(4, d)).standard_normal(seconds * 2048).astype(np.float32)
            for d in range(2)]


def bench_serving(args):
    """128 banks drawn as in the batched workload, 2 detectors, strain pushed in
    1 s strides at `rate` x real time; p50/p99 latency from the push that
    completes a stride to its triggers on the host, and template-samples/s."""
    import torch
    from workloads import configs
    from paper_2410_16416_amd import lloid
    nb = args.banks or 128
    log(f"[bench] serving: generating {nb} banks")
    banks = configs.batched_c3_banks(nb)
    f0 = 2048
    n_strides = args.strides
    xs = serving_inputs()
    torch.cuda.init()
    ctx = lloid.lloid_ctx_create(0)
    out = {}
    sweep = []
    for compute in [args.compute] + (["f32"] if args.f32_steps and args.compute != "f32" else []):
        hs = [lloid.bank_from_svd(ctx, b, compute) for b in banks]
        out[compute] = measure_serving(lloid, ctx, banks, hs, compute, args.rate, n_strides, xs)
        log(f"[bench] serving {compute}: {out[compute]}")
        if compute == args.compute:
            out[compute + "_hip_graph"] = measure_serving(lloid, ctx, banks, hs, compute, args.rate, n_strides, xs,
                                                          use_graph=True)
            log(f"[bench] serving {compute} (HIP graph ticks): {out[compute + '_hip_graph']}")
            out[compute + "_saturation"] = measure_serving(lloid, ctx, banks, hs, compute, 0, n_strides, xs)
            log(f"[bench] serving {compute} at saturation: {out[compute + '_saturation']}")
        if compute == args.compute and args.rates:
            for r in [float(v) for v in args.rates.split(",") if v]:
                sweep.append(measure_serving(lloid, ctx, banks, hs, compute, r, min(1000, int(60 * r)), xs))
                log(f"[bench] serving {compute} at {r:g}x: {sweep[-1]}")
        for h in hs:
            lloid.lloid_bank_destroy(h)
    lloid.lloid_ctx_destroy(ctx)
    m = out[args.compute]
    return {"metric": METRIC, "value": m["value"], "unit": "template-samples/s", "n_gpus": 1,
            "steps": n_strides, "warmup": 4, "ms_per_step": m["ms_per_stride"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.compute,
            "data": "synthetic (seeded white Gaussian noise; uneven bank shapes with seeded random orthonormal bases)",
            "config": {"workload": f"serving_c4: {nb} banks, 2 detectors, 1 s strides at {args.rate:g}x real time",
                       "banks": nb, "templates": sum(b.n_templates for b in banks), "detectors": 2,
                       "strides": n_strides, "rate_x_real_time": args.rate, "f0": f0},
            "p50_stride_latency_ms": m["p50_stride_latency_ms"], "p99_stride_latency_ms": m["p99_stride_latency_ms"],
            "paths": out, "rate_sweep": sweep}


def stated_error(compute: str):
    """The precision's measured SNR error against the FP64 oracle on the
    1024-template bank (recorded by the parity test)."""
    err_path = os.path.join(PROFILES, "precision_multirate_c1.json")
    if not os.path.exists(err_path):
        return None
    with open(err_path) as f:
        return json.load(f).get(compute)


def bench_snr_series(lloid, ctx, wl, xs, args):
    """SNR-series output mode: the complex SNR of every template at every
    sample written to a device buffer [F][n][2] FP32 beside the triggers (8 B
    per template-sample; HBM-bound)."""
    import torch
    F, n = wl.bank.n_templates, wl.n_samples
    log(f"[bench] snr-series mode: steps {args.snr_steps} ({F * n * 8 / 1e9:.1f} GB per detector)")
    dz = torch.empty((F, n, 2), dtype=torch.float32, device="cuda")
    bank = lloid.bank_from_svd(ctx, wl.bank, args.compute)
    try:
        tiles = pick_tiles(lloid, ctx, [bank], args)

        def step():
            for d, x in enumerate(xs):
                lloid.lloid_filter(bank, d, x, window=(1, 1), threshold=4.0, snr_out=dz)
        step()
        torch.cuda.synchronize()
        lloid.lloid_ctx_profile(ctx, True)
        lloid.lloid_ctx_stage_times(ctx, reset=True)
        t0 = time.perf_counter()
        for _ in range(args.snr_steps):
            step()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.snr_steps
        st = lloid.lloid_ctx_stage_times(ctx, reset=True)
        lloid.lloid_ctx_profile(ctx, False)
    finally:
        lloid.lloid_bank_destroy(bank)
        del dz
        torch.cuda.empty_cache()
    ms_mix = st["mix"][0] / max(st["mix"][1], 1)
    series_bytes = F * n * 8
    return {"value": round(F * n * len(xs) / wall, 1), "ms_per_step": round(wall * 1e3, 3),
            "series_bytes_per_detector": series_bytes,
            "mix_ms_per_launch": round(ms_mix, 3),
            "mix_write_gbs": round(series_bytes / (ms_mix / 1e3) / 1e9, 1),
            "hbm_peak_gbs": PEAK_HBM_GBS, "floor_ms_per_step": round(series_bytes * len(xs) / PEAK_HBM_GBS / 1e6, 3),
            "tiles": tiles}


def bench_c0_latency(lloid, ctx, args):
    """Latency of one call on the single-rate 64-template workload (8 s at
    1024 Hz, one detector, 0.1 s windows): host strain in, triggers out."""
    import numpy as np
    from workloads import configs
    wl = configs.plain_c0()
    x = wl.strains[0]
    bank = lloid.bank_from_svd(ctx, wl.bank, args.compute)
    try:
        for _ in range(10):
            lloid.lloid_filter(bank, 0, x, window=(1, 10))
        lat = []
        for _ in range(args.c0_calls):
            t0 = time.perf_counter()
            r = lloid.lloid_filter(bank, 0, x, window=(1, 10))
            lat.append((time.perf_counter() - t0) * 1e3)
    finally:
        lloid.lloid_bank_destroy(bank)
    lat = np.array(lat)
    return {"workload": "plain_c0: 64 chirp templates at 1024 Hz, 32 basis filters, 8 s, 0.1 s windows",
            "calls": args.c0_calls, "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "triggers": int(r.n_triggers),
            "template_samples_per_s_at_p50": round(64 * x.shape[0] / (np.percentile(lat, 50) / 1e3), 1),
            "timing": "host wall time of lloid_filter (host FP64 strain in, triggers in host memory out)"}


def bench_c3_c4(lloid, ctx, args):
    """The batched form (64 uneven banks, 2 detectors x 512 s) and the serving
    form (128 banks streamed in 1 s strides at 16x real time and at
    saturation), the operand type of the headline."""
    import numpy as np
    import torch
    from workloads import configs
    n_banks = 128 if args.c4_strides else 64
    log(f"[bench] generating {n_banks} uneven banks")
    t0 = time.perf_counter()
    banks = configs.batched_c3_banks(n_banks)
    log(f"[bench] banks ready in {time.perf_counter() - t0:.1f} s")
    out = {}
    if args.c3_steps:
        seconds = 512
        c3 = banks[:64]
        xs = [torch.from_numpy(np.random.default_rng(configs.seed(3, d)).standard_normal(seconds * 2048)).to("cuda")
              for d in range(2)]
        saved = args.block_seconds
        args.block_seconds = seconds
        r = measure_batched(lloid, ctx, c3, xs, args.compute, args.c3_steps, 1, seconds, args)
        args.block_seconds = saved
        del xs
        out["batched_c3"] = dict(workload="batched_c3: 64 uneven SVD banks (F U[200,2000], 1-4 slices, filters "
                                          "0.5-64 s), 2 detectors x 512 s, one launch per stage",
                                 templates=sum(b.n_templates for b in c3), **r)
        log(f"[bench] batched_c3: {r['ms_per_step']} ms/step, MFMA fraction {r['mfma_frac_of_peak']}")
    if args.c4_strides:
        xs = serving_inputs()
        hs = [lloid.bank_from_svd(ctx, b, args.compute) for b in banks]
        lloid.lloid_ctx_set_tiles(ctx, 0, 0)   # serving ticks keep the default tiles
        try:
            a = measure_serving(lloid, ctx, banks, hs, args.compute, 16.0, args.c4_strides, xs)
            log(f"[bench] serving_c4 16x: {a}")
            b = measure_serving(lloid, ctx, banks, hs, args.compute, 0, args.c4_strides, xs)
            log(f"[bench] serving_c4 saturation: {b}")
        finally:
            for h in hs:
                lloid.lloid_bank_destroy(h)
        out["serving_c4"] = {"workload": "serving_c4: 128 uneven banks, 2 detectors, 1 s strides, max 2 windows "
                                         "per tick, default tiles",
                             "templates": sum(b.n_templates for b in banks), "at_16x": a, "at_saturation": b}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--compute", default="f16", choices=["f16", "bf16", "f32"])
    ap.add_argument("--seconds", type=int, default=1024, help="seconds of strain per detector")
    ap.add_argument("--f32-steps", type=int, default=3, help="timed steps of the plain FP32 path (0: skip)")
    ap.add_argument("--cpu-sample-s", type=float, default=60.0,
                    help="seconds of outputs per oracle process (0: skip the CPU baseline)")
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="single-threaded oracle processes, one per host core (at most 16)")
    ap.add_argument("--bf16-steps", type=int, default=3, help="timed steps of the BF16 path (0: skip)")
    ap.add_argument("--snr-steps", type=int, default=2,
                    help="timed steps of the SNR-series output mode (complex SNR of every template and "
                         "sample written to HBM; 0: skip)")
    ap.add_argument("--c0-calls", type=int, default=100, help="timed calls of the 64-template single-rate "
                                                              "block (latency; 0: skip)")
    ap.add_argument("--c3-steps", type=int, default=2, help="default run: timed steps of the 64 uneven banks "
                                                            "(2 detectors x 512 s; 0: skip)")
    ap.add_argument("--c4-strides", type=int, default=200, help="default run: timed 1 s strides of the 128-bank "
                                                                "serving stream at 16x and at saturation (0: skip)")
    ap.add_argument("--workload", default="multirate_c1", choices=["multirate_c1", "batched_c3", "serving_c4"],
                    help="multirate_c1 (headline), batched_c3 (64 uneven banks, one launch per stage), "
                         "serving_c4 (128 banks streamed in 1 s strides)")
    ap.add_argument("--banks", type=int, default=0, help="banks for batched_c3 / serving_c4 (0: 64 / 128)")
    ap.add_argument("--rate", type=float, default=16.0, help="serving_c4: strides per second (x real time)")
    ap.add_argument("--rates", default="", help="serving_c4: also sweep these rates (e.g. 1,4,16,64), "
                                                "min(1000, 60 x rate) strides each, operand type only")
    ap.add_argument("--strides", type=int, default=120, help="serving_c4: timed 1 s strides")
    ap.add_argument("--xi2-half", type=int, default=175,
                    help="multirate_c1: lags K on each side of the signal-consistency path (2K + 1 samples)")
    ap.add_argument("--xi2-steps", type=int, default=3, help="timed steps of the path with xi2 (0: skip)")
    ap.add_argument("--coinc-reps", type=int, default=5, help="timed coincidence calls on the last triggers (0: skip)")
    ap.add_argument("--cond-reps", type=int, default=5, help="timed conditioning calls on one detector (0: skip)")
    ap.add_argument("--tune-seconds", type=float, default=-1.0,
                    help="autotuning of the tile shapes on this much synthetic strain when the cache has no "
                         "choice for the banks (-1: the workload's block length; 0: default tiles)")
    ap.add_argument("--tile-cache", default=TILE_CACHE, help="JSON record of autotuned tile shapes")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (PMC byte-counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the filtering path runs on a single MI355X "
              "(sharding by bank over several GPUs is not run here)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from workloads import configs
    from paper_2410_16416_amd import lloid

    if args.workload == "batched_c3":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.workload == "serving_c4":
        print(json.dumps(bench_serving(args)), flush=True)
        return
    log(f"[bench] generating workload ({args.seconds} s x 2 detectors)")
    t0 = time.perf_counter()
    wl = configs.multirate_c1(seconds=args.seconds)
    args.block_seconds = args.seconds
    log(f"[bench] workload ready in {time.perf_counter() - t0:.1f} s: {wl.bank.describe()}")
    cpu = cpu1 = None
    if args.cpu_sample_s > 0:
        # before the GPU is initialised: spawned single-threaded oracle processes
        log(f"[bench] cpu baseline: {args.cpu_workers} oracle processes x {args.cpu_sample_s:g} s")
        cpu = cpu_baseline(wl, args.cpu_sample_s, args.cpu_workers)
        cpu1 = cpu_baseline_1thread(wl, 4.0)
        log(f"[bench] cpu baseline: {cpu['value']:.4g} template-samples/s on {cpu['cores']} processes")
    torch.cuda.init()
    ctx = lloid.lloid_ctx_create(0)
    xs = [torch.from_numpy(x).to("cuda") for x in wl.strains]
    n_win = -(-wl.n_samples // wl.bank.f0)
    cap = wl.bank.n_templates * n_win
    tbufs = [torch.empty(cap * lloid.TRIGGER_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True) for _ in xs]
    torch.cuda.synchronize()

    F, f0 = wl.bank.n_templates, wl.bank.f0
    samples_per_step = F * wl.n_samples * len(xs)
    log(f"[bench] {args.compute}: warmup {args.warmup}, steps {args.steps}")
    wall, n_trig, stages, tiles = run_path(lloid, ctx, wl, xs, args.compute, args.steps, args.warmup, tbufs, args)
    ms_step = wall / args.steps * 1e3
    value = samples_per_step / (wall / args.steps)
    log(f"[bench] {args.compute}: {ms_step:.2f} ms/step, {value:.4g} template-samples/s, stages {stages}")

    work = stage_work(wl.bank, wl.n_samples / f0, args.compute)
    roofs = {}
    for st, (kind, w) in work.items():
        ms, calls = stages[st]
        if calls:
            roofs[st] = roofline_entry(kind, w, ms / calls, args.compute, load_traffic(st, args.compute))
            roofs[st]["ms_per_launch"] = round(ms / calls, 4)
    dominant = max(roofs, key=lambda k: roofs[k]["ms_per_launch"])

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "template-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.compute,
        "data": "synthetic (seeded white Gaussian noise + chirp injections; closed-form chirp bank)",
        "config": {"workload": "multirate_c1: 1024 chirp templates (0.5-32 s), slices 2048/512/128 Hz "
                               "with 200/150/100 basis filters, 2 detectors x 1024 s, 20 injections, "
                               "1 s windows, threshold 4",
                   "templates": F, "detectors": len(xs), "seconds": wl.n_samples // f0, "f0": f0,
                   "compute": args.compute, "accumulate": "f32"},
        "templates_in_real_time": round(value / f0, 1),
        "triggers_per_step": int(n_trig),
        "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stages.items()},
        "roofline": dict(roofs[dominant], kernel=dominant),
        "tiles": tiles,
        "roofline_stages": roofs,
        "p99_stride_latency_ms": None,
    }
    out["stated_snr_error"] = stated_error(args.compute)

    if args.f32_steps and args.compute != "f32":
        log(f"[bench] plain f32 path: steps {args.f32_steps}")
        w32, _, st32, _ = run_path(lloid, ctx, wl, xs, "f32", args.f32_steps, 1, tbufs, args)
        v32 = samples_per_step / (w32 / args.f32_steps)
        ms, calls = st32["mix"]
        out["f32_path"] = {"value": round(v32, 1), "ms_per_step": round(w32 / args.f32_steps * 1e3, 3),
                           "speedup_of_headline": round(value / v32, 2),
                           "roofline_mix": roofline_entry("mfma", work["mix"][1], ms / max(calls, 1), "f32")}
    if args.cond_reps:
        # conditioning of one detector's block (PSD estimate, whitening, gating)
        # from and to HBM, 2 s segments
        L = 4096
        dout = torch.empty(wl.n_samples, dtype=torch.float32, device="cuda")
        lloid.lloid_condition(ctx, f0, xs[0], L, gate_threshold=50.0, gate_half_width=512, out=dout)
        torch.cuda.synchronize()
        t0c = time.perf_counter()
        for _ in range(args.cond_reps):
            _, _, n_gated = lloid.lloid_condition(ctx, f0, xs[0], L, gate_threshold=50.0, gate_half_width=512,
                                                  out=dout)
        torch.cuda.synchronize()
        msc = (time.perf_counter() - t0c) / args.cond_reps * 1e3
        out["conditioning"] = {"seg_len": L, "samples": wl.n_samples, "ms_per_call": round(msc, 3),
                               "samples_per_s": round(wl.n_samples / msc * 1e3, 1), "gated": n_gated,
                               "timing": "host wall time of the call (device strain in and out)"}
    if args.coinc_reps:
        # coincidence of the two detectors' triggers (same template, within the
        # light travel time: 10 ms, 21 samples at 2048 Hz), lists resident in HBM
        bank = lloid.bank_from_svd(ctx, wl.bank, args.compute)
        try:
            trig = [lloid.lloid_filter(bank, d, x, window=(1, 1), threshold=4.0).triggers for d, x in enumerate(xs)]
        finally:
            lloid.lloid_bank_destroy(bank)
        dev = [torch.from_numpy(t.view(np.uint8).copy()).to("cuda") for t in trig]
        pairs = lloid.lloid_coincide(ctx, dev[0], dev[1], 21)
        torch.cuda.synchronize()
        t0c = time.perf_counter()
        for _ in range(args.coinc_reps):
            pairs = lloid.lloid_coincide(ctx, dev[0], dev[1], 21, cap=pairs.shape[0] + 16)
        torch.cuda.synchronize()
        out["coincidence"] = {"max_dt_samples": 21, "triggers": [int(t.shape[0]) for t in trig],
                              "pairs": int(pairs.shape[0]),
                              "ms_per_call": round((time.perf_counter() - t0c) / args.coinc_reps * 1e3, 3),
                              "timing": "host wall time of the call (device lists, host output)"}
    if args.xi2_steps and args.xi2_half > 0:
        from workloads import bank_autocorrelation
        log(f"[bench] {args.compute} with xi2 over {2 * args.xi2_half + 1} lags: steps {args.xi2_steps}")
        wl.bank.autocorr = bank_autocorrelation(wl.bank, args.xi2_half)
        try:
            wx, ntx, stx, _ = run_path(lloid, ctx, wl, xs, args.compute, args.xi2_steps, 1, tbufs, args)
        finally:
            wl.bank.autocorr = None
        out["xi2_path"] = {"lags": 2 * args.xi2_half + 1, "value": round(samples_per_step / (wx / args.xi2_steps), 1),
                           "ms_per_step": round(wx / args.xi2_steps * 1e3, 3),
                           "phase_stage_ms_per_step": round(stx["phase"][0] / args.xi2_steps, 3),
                           "triggers_per_step": int(ntx)}
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b2 = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b2.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
        del a, b2
    if args.bf16_steps and args.compute != "bf16":
        log(f"[bench] bf16 path: steps {args.bf16_steps}")
        wb, nb16, stb, tb = run_path(lloid, ctx, wl, xs, "bf16", args.bf16_steps, 1, tbufs, args)
        ms, calls = stb["mix"]
        out["bf16_path"] = {"value": round(samples_per_step / (wb / args.bf16_steps), 1),
                            "ms_per_step": round(wb / args.bf16_steps * 1e3, 3), "triggers_per_step": int(nb16),
                            "stage_ms_per_step": {k: round(v[0] / args.bf16_steps, 3) for k, v in stb.items()},
                            "roofline_mix": roofline_entry("mfma", work["mix"][1], ms / max(calls, 1), "bf16"),
                            "stated_snr_error": stated_error("bf16"), "tiles": tb}
    if args.snr_steps:
        out["snr_series_mode"] = bench_snr_series(lloid, ctx, wl, xs, args)
    if args.c0_calls:
        out["c0_latency"] = bench_c0_latency(lloid, ctx, args)
    if args.c3_steps or args.c4_strides:
        out.update(bench_c3_c4(lloid, ctx, args))
        if "serving_c4" in out:
            out["p99_stride_latency_ms"] = out["serving_c4"]["at_16x"]["p99_stride_latency_ms"]
            out["p50_stride_latency_ms"] = out["serving_c4"]["at_16x"]["p50_stride_latency_ms"]
    if cpu:
        out["cpu_baseline"] = cpu
    if cpu1:
        out["cpu_baseline_1_thread"] = cpu1
    lloid.lloid_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
