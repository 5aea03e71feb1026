"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Small cases (seconds of oracle time) compare every complex-SNR sample and
every window peak; the full multi-rate workload (1024 templates, 3 slices,
2 detectors x 1024 s) runs on the GPU in the benchmark's launch
configuration and is compared on sampled windows the oracle computes one
by one.
"""

import functools

import numpy as np
import pytest

import oracle
from workloads import configs
from workloads.strain import Injection, inject

from gpu_util import EPS_ABS, compare_peaks, compare_series, ctx, gpu_complex, log, record_precision, run_filter

pytestmark = pytest.mark.gpu
PRECISIONS = ["f32", "f16", "bf16"]


@functools.lru_cache(maxsize=None)
def c0_case():
    wl = configs.plain_c0()
    x = wl.strains[0]
    z = oracle.lloid_snr(wl.bank, x)
    wins, pa, ps, ph = oracle.peak_table(z, 0, 1024, 1, 10)
    return wl, x, z, pa, ps, ph


@functools.lru_cache(maxsize=None)
def mini_case():
    wl = configs.mini_multirate(seconds=12, n_injections=2)
    x = wl.strains[0][: 12 * 1024 - 333]          # ragged tail: not a multiple of any tile
    z = oracle.lloid_snr(wl.bank, x)
    wins, pa, ps, ph = oracle.peak_table(z, 0, 1024, 1, 4)
    return wl, x, z, pa, ps, ph


@pytest.mark.parametrize("compute", PRECISIONS)
def test_c0_series_and_peaks(compute):
    log(f"[c0] compute={compute}")
    wl, x, z, pa, ps, ph = c0_case()
    res = run_filter(wl.bank, x, compute, (1, 10), snr=True)
    zg = gpu_complex(res)
    s = compare_series(zg, z, compute, f"c0/{compute}")
    p = compare_peaks(res, np.abs(z), pa, ps, compute, label=f"c0/{compute}", eps_series=s["max_abs"])
    log(f"  series {s} peaks {p}")
    inj = wl.injections[0]
    assert res.peak_sample[inj.template, 40] == 4146
    assert abs(res.peak_snr[inj.template, 40] - pa[inj.template, 40]) <= EPS_ABS[compute]
    # phase at the peak: compare where the peak sample agrees and |z| is well above the noise
    ok = (res.peak_sample == ps) & (pa >= 4.0)
    dphi = np.angle(np.exp(1j * (res.peak_phase[ok] - ph[ok])))
    assert np.max(np.abs(dphi)) <= 3 * EPS_ABS[compute] / 4.0


@pytest.mark.parametrize("compute", PRECISIONS)
def test_mini_multirate_ragged(compute):
    """Three slices at 1024/256/64 Hz (levels 0, 2, 4 with empty levels between),
    a ragged length and 0.25 s windows."""
    log(f"[mini] compute={compute}")
    wl, x, z, pa, ps, ph = mini_case()
    res = run_filter(wl.bank, x, compute, (1, 4), snr=True)
    s = compare_series(gpu_complex(res), z, compute, f"mini/{compute}")
    p = compare_peaks(res, np.abs(z), pa, ps, compute, label=f"mini/{compute}", eps_series=s["max_abs"])
    log(f"  series {s} peaks {p}")


def test_sigma2_fp64():
    from paper_2410_16416_amd import lloid
    for bank in (configs.plain_c0_bank(), configs.mini_multirate_bank()):
        b = lloid.bank_from_svd(ctx(), bank, "f16")
        try:
            s2 = lloid.lloid_bank_sigma2(b)
        finally:
            lloid.lloid_bank_destroy(b)
        assert np.allclose(s2, oracle.sigma2(bank), rtol=1e-13, atol=0)


def test_triggers_are_thresholded_peaks_and_truncate():
    from paper_2410_16416_amd import lloid
    wl, x, z, pa, ps, ph = c0_case()
    b = lloid.bank_from_svd(ctx(), wl.bank, "f16")
    try:
        res = lloid.lloid_filter(b, 3, x, window=(1, 10), threshold=4.0, peaks=True)
        want = [(i, w) for i in range(res.peak_snr.shape[0]) for w in range(res.peak_snr.shape[1])
                if res.peak_snr[i, w] >= 4.0]
        got = list(zip(res.triggers["template_id"].tolist(), res.triggers["window"].tolist()))
        assert got == want and res.n_triggers == len(want)
        t = res.triggers
        assert np.all(t["detector"] == 3)
        assert np.array_equal(t["sample"], res.peak_sample[t["template_id"], t["window"]])
        assert np.array_equal(t["snr"], res.peak_snr[t["template_id"], t["window"]])
        small = np.empty(5, dtype=lloid.TRIGGER_DTYPE)
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_filter(b, 3, x, window=(1, 10), trig_cap=5, triggers_out=small)
        assert ei.value.status == lloid.LLOID_ETRUNC
        assert np.array_equal(small, res.triggers[:5])
        # a higher threshold keeps exactly the peaks above it
        hi = lloid.lloid_filter(b, 3, x, window=(1, 10), threshold=9.0)
        assert hi.n_triggers == int((res.peak_snr >= 9.0).sum())
    finally:
        lloid.lloid_bank_destroy(b)


def test_triggers_into_pinned_and_device_buffers():
    """A trigger buffer in pinned host memory or in device memory takes the
    records straight from the compaction kernel (no staging copy): the same
    records as a pageable buffer, and a too-small pinned buffer still gets
    ETRUNC with the first records and the required count."""
    import torch
    from paper_2410_16416_amd import lloid
    wl, x, z, pa, ps, ph = mini_case()
    b = lloid.bank_from_svd(ctx(), wl.bank, "f16")
    isz = lloid.TRIGGER_DTYPE.itemsize
    try:
        want = lloid.lloid_filter(b, 0, x, window=(1, 4), threshold=3.0).triggers
        assert want.shape[0] > 20
        cap = want.shape[0] + 7
        pinned = torch.zeros(cap * isz, dtype=torch.uint8, pin_memory=True)
        r = lloid.lloid_filter(b, 0, x, window=(1, 4), threshold=3.0, triggers_out=pinned)
        got = pinned.numpy().view(lloid.TRIGGER_DTYPE)[: r.n_triggers]
        assert r.n_triggers == want.shape[0] and np.array_equal(got, want)
        dev = torch.zeros(cap * isz, dtype=torch.uint8, device="cuda")
        r = lloid.lloid_filter(b, 0, x, window=(1, 4), threshold=3.0, triggers_out=dev)
        torch.cuda.synchronize()
        got = dev.cpu().numpy().view(lloid.TRIGGER_DTYPE)[: r.n_triggers]
        assert r.n_triggers == want.shape[0] and np.array_equal(got, want)
        small = torch.zeros(5 * isz, dtype=torch.uint8, pin_memory=True)
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_filter(b, 0, x, window=(1, 4), threshold=3.0, trig_cap=5, triggers_out=small)
        assert ei.value.status == lloid.LLOID_ETRUNC
        assert np.array_equal(small.numpy().view(lloid.TRIGGER_DTYPE), want[:5])
    finally:
        lloid.lloid_bank_destroy(b)


def test_deterministic_and_device_strain():
    import torch
    from paper_2410_16416_amd import lloid
    wl, x, z, pa, ps, ph = mini_case()
    b = lloid.bank_from_svd(ctx(), wl.bank, "f16")
    try:
        r1 = lloid.lloid_filter(b, 0, x, window=(1, 4), peaks=True)
        r2 = lloid.lloid_filter(b, 0, x, window=(1, 4), peaks=True)
        xd = torch.from_numpy(x).to("cuda")
        torch.cuda.synchronize()
        r3 = lloid.lloid_filter(b, 0, xd, window=(1, 4), peaks=True)
        r4 = lloid.lloid_filter(b, 0, x.astype(np.float32), window=(1, 4), peaks=True)
    finally:
        lloid.lloid_bank_destroy(b)
    for r in (r2, r3):
        assert np.array_equal(r1.peak_snr, r.peak_snr) and np.array_equal(r1.peak_sample, r.peak_sample)
        assert np.array_equal(r1.triggers, r.triggers)
    # FP32 strain input rounds x before conversion: equal within FP16 tolerance
    assert np.max(np.abs(r4.peak_snr - r1.peak_snr)) < EPS_ABS["f16"]


def test_edge_cases_short_inputs_and_errors():
    from paper_2410_16416_amd import lloid
    wl, x, z, pa, ps, ph = c0_case()
    b = lloid.bank_from_svd(ctx(), wl.bank, "f32")
    try:
        for n in (1, 31, 102, 103, 1000):       # shorter than a tile, a window, the filter
            xs = x[:n]
            zo = oracle.lloid_snr(wl.bank, xs)
            _, pao, pso, _ = oracle.peak_table(zo, 0, 1024, 1, 10)
            res = lloid.lloid_filter(b, 0, xs, window=(1, 10), peaks=True)
            assert res.peak_snr.shape == pao.shape
            compare_peaks(res, np.abs(zo), pao, pso, "f32", label=f"n={n}")
        bad = x[:500].copy()
        bad[17] = np.nan
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_filter(b, 0, bad, window=(1, 10))
        assert ei.value.status == lloid.LLOID_EDATA
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_filter(b, 0, x[:0], window=(1, 10))
        assert ei.value.status == lloid.LLOID_EINVAL
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_filter(b, 0, x[:100], window=(1, 10), strain_scale=3.0)
        assert ei.value.status == lloid.LLOID_EINVAL
        # one window whose operand rows exceed what a buffer resource spans
        # (2^31 - 2^24 bytes) is refused before any device work; a block whose
        # whole operand exceeds it in windows of ordinary length is not (the
        # full-size 1024-template runs below are such blocks)
        long = np.zeros((1 << 24) + (1 << 20), dtype=np.float32)
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_filter(b, 0, long, window=(20000, 1))
        assert ei.value.status == lloid.LLOID_EINVAL
    finally:
        lloid.lloid_bank_destroy(b)
    sl = wl.bank.slices[0]

    class S:
        pass
    for rate, start, nb in ((1000, 0, 8), (512, 1, 8), (1024, 0, 2000)):
        s = S()
        s.rate, s.start_tap, s.n_taps = rate, start, sl.n_taps
        s.basis = np.zeros((nb, sl.n_taps)) if nb <= sl.n_taps else np.zeros((nb, sl.n_taps))
        s.mixing = np.zeros((128, nb))
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_bank_create(ctx(), 1024, 64, [s], "f16")
        assert ei.value.status == lloid.LLOID_EINVAL


# ---------------------------------------------------------------- C1 scale

def c1_small_workload(seconds=36):
    bank = configs.multirate_c1_bank()
    wl = configs.multirate_c1(seconds=seconds, detectors=1, n_injections=0, bank=bank)
    injs = [Injection(template=17, t0=33 * 2048 + 611, snr=12.0, phase=0.7),
            Injection(template=900, t0=34 * 2048 + 1500, snr=25.0, phase=-2.0)]
    x = inject(wl.strains[0], bank.family, injs)[: seconds * 2048 - 777]
    return bank, x, injs


@functools.lru_cache(maxsize=None)
def c1_small_case():
    bank, x, injs = c1_small_workload()
    tsel = np.array(sorted({17, 900} | set(range(0, 1024, 37))))
    z = oracle.lloid_snr(bank, x, templates=tsel)
    wins, pa, ps, ph = oracle.peak_table(z, 0, 2048, 1, 1)
    return bank, x, injs, tsel, z, pa, ps


@pytest.mark.parametrize("compute", PRECISIONS)
def test_c1_bank_short_block(compute):
    """The full 1024-template, three-slice bank on 36 s (every slice's history
    filled, ragged end), 1 s windows; series and peaks on a template subset."""
    log(f"[c1-short] compute={compute}")
    bank, x, injs, tsel, z, pa, ps = c1_small_case()
    res = run_filter(bank, x, compute, (1, 1), snr=True)
    zg = gpu_complex(res)[tsel]
    s = compare_series(zg, z, compute, f"c1short/{compute}")
    res.peak_snr, res.peak_sample = res.peak_snr[tsel], res.peak_sample[tsel]
    p = compare_peaks(res, np.abs(z), pa, ps, compute, label=f"c1short/{compute}", eps_series=s["max_abs"])
    log(f"  series {s} peaks {p}")
    record_precision(f"multirate_c1 bank, 36 s block, {len(tsel)} templates, every sample", compute, **s, **p)
    for inj in injs:
        r = int(np.nonzero(tsel == inj.template)[0][0])
        w = inj.t0 // 2048
        # noise moves the argmax of a low-frequency chirp by a few samples
        assert abs(res.peak_sample[r, w] - inj.t0) <= 16
        assert res.peak_snr[r, w] > 0.85 * inj.snr


@functools.lru_cache(maxsize=None)
def c1_full_inputs():
    wl = configs.multirate_c1()
    return wl


@pytest.mark.parametrize("compute", PRECISIONS)
def test_c1_full_size_sampled_windows(compute):
    """2 detectors x 1024 s at the benchmark's launch configuration; the oracle
    recomputes all 1024 templates on sampled 1 s windows (injection windows,
    the first, the last, and random ones)."""
    from paper_2410_16416_amd import lloid
    log(f"[c1-full] compute={compute}")
    wl = c1_full_inputs()
    bank = wl.bank
    b = lloid.bank_from_svd(ctx(), bank, compute)
    rng = np.random.default_rng(11)
    try:
        for det, x in enumerate(wl.strains):
            res = lloid.lloid_filter(b, det, x, window=(1, 1), peaks=True)
            assert res.peak_snr.shape == (1024, 1024)
            inj_w = sorted({inj.t0 // 2048 for inj in wl.injections})
            sample = sorted(set(inj_w[:3]) | {0, 1023} | set(rng.integers(0, 1024, 3).tolist()))
            for w in sample:
                z = oracle.lloid_snr(bank, x, w * 2048, (w + 1) * 2048)
                _, pa, ps, _ = oracle.peak_table(z, w * 2048, 2048, 1, 1)

                class R:
                    pass
                r = R()
                r.peak_snr, r.peak_sample = res.peak_snr[:, [w]], res.peak_sample[:, [w]]
                compare_peaks(r, np.abs(z), pa, ps, compute, n_lo=w * 2048, label=f"c1full/{compute}/d{det}/w{w}")
            for inj in wl.injections:
                w = inj.t0 // 2048
                assert res.peak_snr[inj.template, w] > 0.85 * inj.snr
                assert abs(res.peak_sample[inj.template, w] - inj.t0) <= 16
            log(f"  det {det}: {res.n_triggers} triggers, windows checked {sample}")
    finally:
        lloid.lloid_bank_destroy(b)


XI_HALF = 20


@pytest.mark.parametrize("compute", PRECISIONS)
def test_xi2_matches_oracle(compute):
    """Every trigger's signal-consistency value equals the oracle's xi2 from the
    oracle's z at the trigger's peak sample (where that sample agrees with the
    oracle's, i.e. outside near ties).  Bound: with |dz| <= eps on every lag
    (eps the stated complex-SNR tolerance), d_k = z_k - z* R_k moves by at most
    2 eps, so the numerator moves by at most 4 eps sum|d_k| + 4 eps^2 n_lags;
    divided by the denominator.  Chunking (a few windows per chunk, so lags
    cross chunk edges) gives bit-identical records; lags before sample 0 and
    past the data end drop out as in the oracle."""
    from paper_2410_16416_amd import lloid
    from workloads import bank_autocorrelation
    log(f"[xi2] compute={compute}")
    wl, x, z, _, _, _ = mini_case()
    n = x.shape[0]
    r = bank_autocorrelation(wl.bank, XI_HALF)
    wl.bank.autocorr = r
    b = lloid.bank_from_svd(ctx(), wl.bank, compute)
    try:
        res = lloid.lloid_filter(b, 0, x, window=(1, 4), threshold=3.0)
        lloid.lloid_ctx_set_chunk_bytes(ctx(), 400000)
        try:
            chunked = lloid.lloid_filter(b, 0, x, window=(1, 4), threshold=3.0)
        finally:
            lloid.lloid_ctx_set_chunk_bytes(ctx(), 6 << 30)
    finally:
        lloid.lloid_bank_destroy(b)
        wl.bank.autocorr = None
    t = res.triggers
    assert t.shape[0] > 20
    assert np.array_equal(t, chunked.triggers)
    eps = EPS_ABS[compute]
    a = np.abs(z)
    wins = t["window"].astype(np.int64)
    starts = oracle.window_starts(int(wins.max()) + 2, 1024, 1, 4)
    lag = np.arange(-XI_HALF, XI_HALF + 1)
    n_cmp, worst = 0, 0.0
    for rec in t:
        i, s, w = int(rec["template_id"]), int(rec["sample"]), int(rec["window"])
        if a[i, starts[w]:min(starts[w + 1], n)].argmax() + starts[w] != s:
            continue
        want = oracle.xi2(z[i], 0, n, s, r[i])
        ok = (s + lag >= 0) & (s + lag < n)
        d = z[i, (s + lag)[ok]] - z[i, s] * r[i, ok]
        den = np.sum(2.0 - 2.0 * np.abs(r[i, ok]) ** 2)
        tol = (4 * eps * np.sum(np.abs(d)) + 4 * eps ** 2 * ok.sum()) / den + 1e-5 * want
        assert abs(float(rec["xi2"]) - want) <= tol, (i, s, float(rec["xi2"]), want, tol)
        worst = max(worst, abs(float(rec["xi2"]) - want))
        n_cmp += 1
    assert n_cmp > 0.8 * t.shape[0]
    assert np.all(t["xi2"] >= 0)
    log(f"  {t.shape[0]} triggers, {n_cmp} compared, max |d xi2| {worst:.2e}")


@pytest.mark.parametrize("compute", ["f16", "f32"])
def test_xi2_more_triggers_than_one_list_pass(compute):
    """A window with more triggers than the kernel lists at once (threshold 0:
    every one of 1500 templates triggers in every window) is handled in
    several passes over the templates (16-bit: the listing stores the passes'
    sorted runs one after the other and the tile launch takes units of 64 that
    can straddle two runs); every value still matches the oracle."""
    from paper_2410_16416_amd import lloid
    from workloads import SliceSpec, bank_autocorrelation
    rng = np.random.default_rng(71)
    bank = configs.random_basis_bank(1500, [SliceSpec(1024, 0, 96, 12), SliceSpec(256, 96, 40, 8)], 1024, rng)
    half = 6
    r = bank_autocorrelation(bank, half)
    bank.autocorr = r
    x = rng.standard_normal(3 * 1024 + 77)
    n = x.shape[0]
    log(f"[xi2 passes] compute={compute}")
    h = lloid.bank_from_svd(ctx(), bank, compute)
    try:
        t = lloid.lloid_filter(h, 0, x, window=(1, 1), threshold=0.0).triggers
    finally:
        lloid.lloid_bank_destroy(h)
    assert t.shape[0] == 1500 * 4
    z = oracle.lloid_snr(bank, x)
    a = np.abs(z)
    starts = oracle.window_starts(5, 1024, 1, 1)
    worst, n_cmp = 0.0, 0
    for rec in t:
        i, s_, w = int(rec["template_id"]), int(rec["sample"]), int(rec["window"])
        if a[i, starts[w]:min(starts[w + 1], n)].argmax() + starts[w] != s_:
            continue
        want = oracle.xi2(z[i], 0, n, s_, r[i])
        lag = np.arange(-half, half + 1)
        ok = (s_ + lag >= 0) & (s_ + lag < n)
        d = z[i, (s_ + lag)[ok]] - z[i, s_] * r[i, ok]
        den = np.sum(2.0 - 2.0 * np.abs(r[i, ok]) ** 2)
        eps = EPS_ABS[compute]   # the bound of test_xi2_matches_oracle
        tol = (4 * eps * np.sum(np.abs(d)) + 4 * eps ** 2 * ok.sum()) / den + 1e-5 * want
        assert abs(float(rec["xi2"]) - want) <= tol, (i, w, float(rec["xi2"]), want, tol)
        worst = max(worst, abs(float(rec["xi2"]) - want))
        n_cmp += 1
    log(f"  {t.shape[0]} triggers, {n_cmp} compared, max |d xi2| {worst:.2e}")
    assert n_cmp > 0.95 * t.shape[0]


@functools.lru_cache(maxsize=None)
def c1_autocorr(half: int):
    from workloads import bank_autocorrelation
    return bank_autocorrelation(c1_full_inputs().bank, half)


@pytest.mark.parametrize("compute", ["f16", "bf16"])
def test_c1_full_size_trigger_fields_sampled(compute):
    """The benchmark's signal-consistency configuration at full size: the
    1024-template bank with 351 lags (K = 175; 480 concatenated columns, so
    the tile launch's 32-step form), detector 0 x 1024 s in one call.  Sampled
    triggers (up to 12 from each of the injection windows, the first, the
    last and random windows) against the oracle's z of the trigger's template
    around its peak, outside near ties: xi2 with the bound of
    test_xi2_matches_oracle; the sub-sample refinement with the bounds of
    test_subsample_peaks_match_oracle; the phase within 2 eps / |z*| (the
    angle a complex error of eps can turn)."""
    from paper_2410_16416_amd import lloid
    half = 175
    log(f"[c1-full xi2] compute={compute}")
    wl = c1_full_inputs()
    bank, x = wl.bank, wl.strains[0]
    n = x.shape[0]
    r = c1_autocorr(half)
    bank.autocorr = r
    try:
        b = lloid.bank_from_svd(ctx(), bank, compute)
    finally:
        bank.autocorr = None
    try:
        t = lloid.lloid_filter(b, 0, x, window=(1, 1)).triggers
    finally:
        lloid.lloid_bank_destroy(b)
    assert t.shape[0] > 10000 and np.all(t["xi2"] >= 0)
    rng = np.random.default_rng(13)
    inj_w = sorted({inj.t0 // 2048 for inj in wl.injections})
    wins = sorted(set(inj_w[:3]) | {0, 1023} | set(rng.integers(1, 1023, 3).tolist()))
    eps = EPS_ABS[compute]
    lag = np.arange(-half, half + 1)
    n_cmp, n_pick, worst, worst_phi = 0, 0, 0.0, 0.0
    for w in wins:
        sel = np.flatnonzero(t["window"] == w)
        for k in rng.choice(sel, size=min(12, sel.shape[0]), replace=False):
            rec = t[k]
            i, s_ = int(rec["template_id"]), int(rec["sample"])
            n_pick += 1
            lo = max(0, min(w * 2048, s_ - half))
            hi = min(n, max((w + 1) * 2048, s_ + half + 1))
            z = oracle.lloid_snr(wl.bank, x, lo, hi, templates=np.array([i]))[0]
            a = np.abs(z[w * 2048 - lo:min((w + 1) * 2048, n) - lo])
            if a.argmax() + w * 2048 != s_:
                continue   # near tie: the GPU's peak is another sample
            want = oracle.xi2(z, lo, n, s_, r[i])
            ok = (s_ + lag >= 0) & (s_ + lag < n)
            d = z[(s_ + lag)[ok] - lo] - z[s_ - lo] * r[i, ok]
            den = np.sum(2.0 - 2.0 * np.abs(r[i, ok]) ** 2)
            tol = (4 * eps * np.sum(np.abs(d)) + 4 * eps ** 2 * ok.sum()) / den + 1e-5 * want
            assert abs(float(rec["xi2"]) - want) <= tol, (i, w, s_, float(rec["xi2"]), want, tol)
            worst = max(worst, abs(float(rec["xi2"]) - want))
            # sub-sample refinement and phase from the same oracle z
            am, a0, ap = (float(abs(z[s_ + k - lo])) for k in (-1, 0, 1))
            dt_o, v_o = oracle.subsample_peak(np.array([am]), np.array([a0]), np.array([ap]))
            assert abs(float(rec["snr_interp"]) - float(v_o[0])) <= 2 * eps, (i, w, s_)
            curv = am - 2.0 * a0 + ap
            assert abs(float(rec["dt"]) - float(dt_o[0])) <= min(1.0, 4 * eps / max(abs(curv), 1e-12)) + 1e-6
            dphi = np.angle(np.exp(1j * (float(rec["phase"]) - np.angle(z[s_ - lo]))))
            assert abs(dphi) <= 2 * eps / a0 + 1e-5, (i, w, s_, float(rec["phase"]), np.angle(z[s_ - lo]))
            worst_phi = max(worst_phi, abs(dphi))
            n_cmp += 1
    log(f"  {t.shape[0]} triggers; windows {wins}: {n_cmp} of {n_pick} sampled compared, max |d xi2| {worst:.2e}, "
        f"max |d phase| {worst_phi:.2e}")
    assert n_cmp > 0.8 * n_pick and n_cmp >= 40


LONG_BASES = {288: [(1024, 0, 160, 128), (256, 160, 96, 96), (64, 544, 80, 64)],
              544: [(1024, 0, 288, 256), (256, 288, 200, 192), (64, 1088, 100, 96)]}


@pytest.mark.parametrize("compute,kcat", [("f16", 288), ("f32", 288), ("f16", 544), ("bf16", 544)])
def test_xi2_long_concatenated_basis(compute, kcat):
    """Banks with long concatenated bases (threshold 0: every template
    triggers in every window), every trigger's value against the oracle.
    kcat 288: 18 16-bit k-steps run in the tile launch's 32-step form (k-steps
    18..31 multiply zeros); FP32 takes 144 k-steps in the one-launch kernel's
    blocks of 10 with a partial last block.  kcat 544: 34 16-bit k-steps, more
    than the tile launch holds in registers, so 16-bit operands take the
    one-launch kernel too."""
    from paper_2410_16416_amd import lloid
    from workloads import SliceSpec, bank_autocorrelation
    rng = np.random.default_rng(73)
    log(f"[xi2 long K] compute={compute} kcat={kcat}")
    specs = [SliceSpec(*sp) for sp in LONG_BASES[kcat]]
    bank = configs.random_basis_bank(200, specs, 1024, rng)
    half = 24
    r = bank_autocorrelation(bank, half)
    bank.autocorr = r
    x = rng.standard_normal(6 * 1024 + 301)
    n = x.shape[0]
    h = lloid.bank_from_svd(ctx(), bank, compute)
    try:
        assert lloid.lloid_bank_query(h).concat_k == kcat
        t = lloid.lloid_filter(h, 0, x, window=(1, 1), threshold=0.0).triggers
    finally:
        lloid.lloid_bank_destroy(h)
    assert t.shape[0] == 200 * 7
    z = oracle.lloid_snr(bank, x)
    a = np.abs(z)
    starts = oracle.window_starts(7, 1024, 1, 1)
    worst, n_cmp = 0.0, 0
    for rec in t:
        i, s_, w = int(rec["template_id"]), int(rec["sample"]), int(rec["window"])
        if a[i, starts[w]:min(starts[w + 1], n)].argmax() + starts[w] != s_:
            continue
        want = oracle.xi2(z[i], 0, n, s_, r[i])
        lag = np.arange(-half, half + 1)
        ok = (s_ + lag >= 0) & (s_ + lag < n)
        d = z[i, (s_ + lag)[ok]] - z[i, s_] * r[i, ok]
        den = np.sum(2.0 - 2.0 * np.abs(r[i, ok]) ** 2)
        eps = EPS_ABS[compute]   # the bound of test_xi2_matches_oracle
        tol = (4 * eps * np.sum(np.abs(d)) + 4 * eps ** 2 * ok.sum()) / den + 1e-5 * want
        assert abs(float(rec["xi2"]) - want) <= tol, (i, w, float(rec["xi2"]), want, tol)
        worst = max(worst, abs(float(rec["xi2"]) - want))
        n_cmp += 1
    log(f"  {t.shape[0]} triggers, {n_cmp} compared, max |d xi2| {worst:.2e}")
    assert n_cmp > 0.9 * t.shape[0]


@pytest.mark.parametrize("compute", PRECISIONS)
def test_subsample_peaks_match_oracle(compute):
    """Every trigger's sub-sample refinement equals the oracle's parabola through
    the oracle's |z| at the peak sample and its neighbours (where the peak sample
    agrees, i.e. outside near ties), and does not depend on chunking: forcing
    chunks of a few windows gives bit-identical records."""
    from paper_2410_16416_amd import lloid
    log(f"[subsample] compute={compute}")
    wl, x, _, _, _, _ = mini_case()
    n = x.shape[0]
    z = oracle.lloid_snr(wl.bank, x, -1, n + 1)          # one sample of margin on each side
    a = np.abs(z)
    b = lloid.bank_from_svd(ctx(), wl.bank, compute)
    try:
        res = lloid.lloid_filter(b, 0, x, window=(1, 4), threshold=3.0)
        lloid.lloid_ctx_set_chunk_bytes(ctx(), 400000)
        try:
            chunked = lloid.lloid_filter(b, 0, x, window=(1, 4), threshold=3.0)
        finally:
            lloid.lloid_ctx_set_chunk_bytes(ctx(), 6 << 30)
    finally:
        lloid.lloid_bank_destroy(b)
    t = res.triggers
    assert t.shape[0] > 20
    assert np.array_equal(t, chunked.triggers)
    eps = EPS_ABS[compute]
    i, s = t["template_id"].astype(np.int64), t["sample"].astype(np.int64)
    dt_o, v_o = oracle.subsample_peak(a[i, s], a[i, s + 1], a[i, s + 2])    # a[:, k] is sample k - 1
    curv = a[i, s] - 2.0 * a[i, s + 1] + a[i, s + 2]
    # compare where the oracle has the same peak sample (outside near ties)
    wins = t["window"].astype(np.int64)
    starts = oracle.window_starts(int(wins.max()) + 2, 1024, 1, 4)
    same = np.array([a[ii, 1 + starts[w]:1 + min(starts[w + 1], n)].argmax() + starts[w] == ss
                     for ii, w, ss in zip(i, wins, s)])
    assert same.mean() > 0.8
    assert np.all(np.abs(t["snr_interp"][same] - v_o[same]) <= 2 * eps)
    # dt is ill-conditioned where the peak is flat: a perturbation eps of the
    # three values moves the vertex by about 2 eps / |curvature|
    tol = np.minimum(1.0, 4 * eps / np.maximum(np.abs(curv[same]), 1e-12)) + 1e-6
    assert np.all(np.abs(t["dt"][same] - dt_o[same]) <= tol)
    assert np.all(np.abs(t["dt"]) <= 0.5) and np.all(t["snr_interp"] >= t["snr"] - 2 * eps)
    log(f"  {t.shape[0]} triggers, {int(same.sum())} compared, max |d snr_interp| "
        f"{float(np.abs(t['snr_interp'][same] - v_o[same]).max()):.2e}")
