"""Batched filtering: many uneven banks in one launch per stage.

Each bank's peaks and triggers in a batch must equal those of the bank alone,
bit for bit (every output is accumulated in the same order whatever the tile,
chunk or batch it lands in), and must match the FP64 oracle.
"""

import functools

import numpy as np
import pytest

import oracle
from workloads import configs

from gpu_util import EPS_ABS, compare_peaks, ctx, log

pytestmark = pytest.mark.gpu


def test_small_uneven_banks_match_oracle_in_a_batch():
    from paper_2410_16416_amd import lloid
    banks = [configs.small_uneven_bank(i) for i in range(6)]
    log("[batch] " + " | ".join(b.describe() for b in banks))
    rng = np.random.default_rng(17)
    n = 6 * 1024 + 333
    x = rng.standard_normal(n)
    handles = [lloid.bank_from_svd(ctx(), b, "f16") for b in banks]
    try:
        res = lloid.lloid_filter_batch(handles, 1, x, window=(1, 4), peaks=True)
        alone = [lloid.lloid_filter(h, 1, x, window=(1, 4), peaks=True) for h in handles]
    finally:
        for h in handles:
            lloid.lloid_bank_destroy(h)
    for k, b in enumerate(banks):
        z = oracle.lloid_snr(b, x)
        _, pa, ps, _ = oracle.peak_table(z, 0, b.f0, 1, 4)

        class R:
            pass
        r = R()
        r.peak_snr, r.peak_sample = res.peak_snr[k], res.peak_sample[k]
        compare_peaks(r, np.abs(z), pa, ps, "f16", label=f"bank{k}")
        assert np.array_equal(res.peak_snr[k], alone[k].peak_snr)
        assert np.array_equal(res.peak_sample[k], alone[k].peak_sample)
        assert np.array_equal(res.peak_phase[k], alone[k].peak_phase)
    # triggers: bank-major, each bank's block equal to its own call (bank field aside)
    t = res.triggers
    assert np.all(np.diff(t["bank"]) >= 0)
    for k in range(len(banks)):
        mine = t[t["bank"] == k]
        other = alone[k].triggers.copy()
        other["bank"] = k
        assert np.array_equal(mine, other)


def test_batch_chunking_is_invisible():
    """A tiny chunk budget forces many chunks; the results must not change."""
    from paper_2410_16416_amd import lloid
    banks = [configs.small_uneven_bank(i) for i in range(3)]
    x = np.random.default_rng(5).standard_normal(9 * 1024)
    handles = [lloid.bank_from_svd(ctx(), b, "f32") for b in banks]
    try:
        big = lloid.lloid_filter_batch(handles, 0, x, window=(1, 4), peaks=True)
        lloid.lloid_ctx_set_chunk_bytes(ctx(), 200_000)
        small = lloid.lloid_filter_batch(handles, 0, x, window=(1, 4), peaks=True)
    finally:
        lloid.lloid_ctx_set_chunk_bytes(ctx(), 6 << 30)
        for h in handles:
            lloid.lloid_bank_destroy(h)
    for k in range(len(banks)):
        assert np.array_equal(big.peak_snr[k], small.peak_snr[k])
        assert np.array_equal(big.peak_sample[k], small.peak_sample[k])
    assert np.array_equal(big.triggers, small.triggers)


@pytest.mark.parametrize("compute", ["f16", "f32"])
def test_batch_signal_consistency_of_mixed_banks(compute):
    """A batch whose banks 0 and 2 carry autocorrelations and bank 1 does
    not: the signal-consistency launches take the jobs of two banks (units of
    both in one list), in forced small chunks too; every bank's triggers,
    xi2 included, equal that bank filtered alone, and bank 1's xi2 is 0."""
    from paper_2410_16416_amd import lloid
    from workloads import bank_autocorrelation
    banks = [configs.small_uneven_bank(i) for i in range(3)]
    for k in (0, 2):
        banks[k].autocorr = bank_autocorrelation(banks[k], 12)
    x = np.random.default_rng(9).standard_normal(9 * 1024 + 211)
    log(f"[batch xi2] {compute}: " + " | ".join(b.describe() for b in banks))
    handles = [lloid.bank_from_svd(ctx(), b, compute) for b in banks]
    try:
        alone = [lloid.lloid_filter(h, 0, x, window=(1, 4), threshold=3.0).triggers for h in handles]
        for budget in (6 << 30, 200_000):
            lloid.lloid_ctx_set_chunk_bytes(ctx(), budget)
            t = lloid.lloid_filter_batch(handles, 0, x, window=(1, 4), threshold=3.0).triggers
            for k in range(3):
                got = t[t["bank"] == k]
                want = alone[k]
                assert got.shape[0] == want.shape[0] and got.shape[0] > 5, (budget, k)
                for f in want.dtype.names:
                    if f != "bank":
                        assert np.array_equal(got[f], want[f]), (budget, k, f)
            assert np.all(t["xi2"][t["bank"] == 1] == 0) and np.all(t["xi2"][t["bank"] != 1] > 0)
    finally:
        lloid.lloid_ctx_set_chunk_bytes(ctx(), 6 << 30)
        for h in handles:
            lloid.lloid_bank_destroy(h)
        for k in (0, 2):
            banks[k].autocorr = None


def test_c3_shaped_banks_alone_equal_in_batch():
    """Eight banks of the batched recipe's shapes (uneven F, 1-4 slices, up to
    64 s filters), 70 s of strain: batch == alone bit for bit."""
    from paper_2410_16416_amd import lloid
    banks = configs.batched_c3_banks(8)
    log("[c3] " + " | ".join(b.describe() for b in banks))
    x = np.random.default_rng(8).standard_normal(70 * 2048)
    handles = [lloid.bank_from_svd(ctx(), b, "f16") for b in banks]
    try:
        res = lloid.lloid_filter_batch(handles, 0, x, window=(1, 1), peaks=True)
        for k, h in enumerate(handles):
            one = lloid.lloid_filter(h, 0, x, window=(1, 1), peaks=True)
            assert np.array_equal(res.peak_snr[k], one.peak_snr), k
            assert np.array_equal(res.peak_sample[k], one.peak_sample), k
    finally:
        for h in handles:
            lloid.lloid_bank_destroy(h)


@pytest.mark.parametrize("compute", ["f16", "bf16", "f32"])
def test_tile_variants_give_identical_results(compute):
    """Every compiled tile shape of the FIR and mixing kernels (including the
    FIR's Hankel fragment window) gives the same
    triggers and peaks, bit for bit: each output's sum over K runs in the same
    order whatever the tile."""
    from paper_2410_16416_amd import lloid
    banks = [configs.small_uneven_bank(i) for i in range(4)]
    x = np.random.default_rng(6).standard_normal(6 * 1024 + 333)
    c = lloid.lloid_ctx_create(0)
    handles = [lloid.bank_from_svd(c, b, compute) for b in banks]
    try:
        # quarter-second windows: one column tile each; 0.75 s: three, with a
        # ragged last window (odd and even chunk counts per window)
        for window in ((1, 4), (3, 4)):
            ref = None
            for fv in range(lloid.FIR_VARIANTS):
                for mv in range(lloid.MIX_VARIANTS):
                    lloid.lloid_ctx_set_tiles(c, fv, mv)
                    assert lloid.lloid_ctx_get_tiles(c) == (fv, mv)
                    r = lloid.lloid_filter_batch(handles, 0, x, window=window, threshold=3.0, peaks=True)
                    if ref is None:
                        ref = r
                        assert r.n_triggers > 0
                        continue
                    assert np.array_equal(r.triggers, ref.triggers), (window, fv, mv)
                    for k in range(len(banks)):
                        assert np.array_equal(r.peak_snr[k], ref.peak_snr[k]), (window, fv, mv, k)
                        assert np.array_equal(r.peak_sample[k], ref.peak_sample[k]), (window, fv, mv, k)
        # the complex SNR series too (the kernels' series-writing forms)
        series = None
        for mv in range(lloid.MIX_VARIANTS):
            lloid.lloid_ctx_set_tiles(c, 0, mv)
            r = lloid.lloid_filter(handles[0], 0, x, window=(3, 4), threshold=3.0,
                                   snr_out=np.zeros((banks[0].n_templates, x.size, 2), np.float32))
            if series is None:
                series = r.snr
            else:
                assert np.array_equal(r.snr, series), mv
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_ctx_set_tiles(c, lloid.FIR_VARIANTS, 0)
        assert ei.value.status == lloid.LLOID_EINVAL
    finally:
        for h in handles:
            lloid.lloid_bank_destroy(h)
        lloid.lloid_ctx_destroy(c)


def test_autotune_picks_the_fastest_and_caches(tmp_path):
    """The autotuner times every variant pair, keeps the fastest on the
    context and records it; a new context with the same banks takes the
    recorded choice without timing."""
    from paper_2410_16416_amd import lloid
    banks = [configs.small_uneven_bank(i) for i in range(3)]
    cache = str(tmp_path / "tiles.json")
    c = lloid.lloid_ctx_create(0)
    handles = [lloid.bank_from_svd(c, b, "f16") for b in banks]
    try:
        best, res = lloid.lloid_autotune(c, handles, 4.0, cache)
        log(f"[autotune] best {best}; " + ", ".join(f"{r['fir_variant']}/{r['mix_variant']}: {r['ms']:.2f} ms"
                                                   for r in res))
        assert res.shape[0] == lloid.FIR_VARIANTS * lloid.MIX_VARIANTS and np.all(res["ms"] > 0)
        k = int(np.argmin(res["ms"]))
        assert best == (int(res["fir_variant"][k]), int(res["mix_variant"][k]))
        text = open(cache).read()
        assert "f16" in text and f'"fir": {best[0]}, "mix": {best[1]}' in text
    finally:
        for h in handles:
            lloid.lloid_bank_destroy(h)
        lloid.lloid_ctx_destroy(c)
    c2 = lloid.lloid_ctx_create(0)
    handles = [lloid.bank_from_svd(c2, b, "f16") for b in banks]
    try:
        lloid.lloid_ctx_set_tiles(c2, 0, 0)
        again, res2 = lloid.lloid_autotune(c2, handles, 4.0, cache)
        assert res2.shape[0] == 0 and again == best
    finally:
        for h in handles:
            lloid.lloid_bank_destroy(h)
        lloid.lloid_ctx_destroy(c2)


# Banks of the batched measurement's recipe at its real shapes: two drawn
# with real chirp SVD spectra (bank 36: 2000 templates, 2048 + 1024 Hz with
# 208 + 256 basis filters; bank 53: four slices at 2048/1024/512/128 Hz,
# 1899 templates), the longest single-slice filter among the measured banks
# (bank 35: 121456 taps, random orthonormal basis) and the recipe's extreme
# (one 64 s slice of 131072 taps, 400 basis filters, 2000 templates).
C3_SECONDS = 70
C3_WINDOWS = {"bank36": (0, 66, 67), "bank53": (0, 66, 67), "bank35": (66, 67), "longest": (66, 67)}


@functools.lru_cache(maxsize=None)
def c3_parity_case():
    from workloads import Injection, add_waveform, inject
    f0 = 2048
    banks = {"bank36": configs.batched_bank(36), "bank53": configs.batched_bank(53),
             "bank35": configs.batched_c3_bank(35), "longest": configs.longest_c3_bank()}
    x = np.random.default_rng(configs.seed(3, 5)).standard_normal(C3_SECONDS * f0)
    injected = {"bank36": (Injection(11, 66 * f0 + 700, 12.0, 0.7), None),
                "bank53": (Injection(1234, 67 * f0 + 300, 15.0, 2.2), None),
                "bank35": (None, (77, 66 * f0 + 1200, 15.0, 1.1)),
                "longest": (None, (1500, 67 * f0 + 1800, 15.0, 2.0))}
    for name, (inj, rec) in injected.items():
        if inj is not None:
            x = inject(x, banks[name].family, [inj])
        else:
            t, t0, amp, phase = rec
            x = add_waveform(x, amp * configs.reconstructed_waveform(banks[name], t, phase), t0)
    tmpl = {k: (v[0].template if v[0] is not None else v[1][0]) for k, v in injected.items()}
    ref = {}
    for name, b in banks.items():
        for w in C3_WINDOWS[name]:
            z = oracle.lloid_snr(b, x, w * f0, (w + 1) * f0)
            _, pa, ps, _ = oracle.peak_table(z, w * f0, f0, 1, 1)
            ref[name, w] = (z, pa, ps)
    return banks, x, tmpl, ref


@pytest.mark.parametrize("compute", ["f16", "bf16", "f32"])
def test_c3_shaped_banks_match_oracle(compute):
    """The batched form at the batched recipe's real shapes against the FP64
    oracle: every template's 1 s window peaks of the batch call on sampled
    windows (the first, and two with an injection, where the longest filters
    have their whole history), and the complex SNR series of a template subset
    (each bank alone; its peaks equal the batch's bit for bit)."""
    import torch
    from paper_2410_16416_amd import lloid
    from gpu_util import compare_series, record_precision
    banks, x, tmpl, ref = c3_parity_case()
    names = list(banks)
    log(f"[c3-oracle] compute={compute} " + " | ".join(f"{k}: {banks[k].describe()}" for k in names))
    handles = [lloid.bank_from_svd(ctx(), banks[k], compute) for k in names]
    f0, n = 2048, x.shape[0]
    stats = {}
    try:
        res = lloid.lloid_filter_batch(handles, 0, x, window=(1, 1), peaks=True)
        for k, name in enumerate(names):
            F = banks[name].n_templates
            sub = np.unique(np.concatenate([np.arange(0, F, max(1, F // 48)), [tmpl[name]]]))
            snr = torch.zeros((F, n, 2), dtype=torch.float32, device="cuda")
            one = lloid.lloid_filter(handles[k], 0, x, window=(1, 1), peaks=True, snr_out=snr)
            assert np.array_equal(one.peak_snr, res.peak_snr[k]), name
            assert np.array_equal(one.peak_sample, res.peak_sample[k]), name
            wins = C3_WINDOWS[name]
            zg = torch.cat([snr[torch.from_numpy(sub).cuda(), w * f0:(w + 1) * f0] for w in wins], dim=1).cpu().numpy()
            del snr
            zg = zg[..., 0].astype(np.float64) + 1j * zg[..., 1].astype(np.float64)
            zo = np.concatenate([ref[name, w][0][sub] for w in wins], axis=1)
            s = compare_series(zg, zo, compute, f"c3/{name}/{compute}")
            peaks = {"max_abs_peak": 0.0, "near_ties": 0, "windows": 0}
            for w in wins:
                z, pa, ps = ref[name, w]

                class R:
                    pass
                r = R()
                r.peak_snr, r.peak_sample = res.peak_snr[k][:, [w]], res.peak_sample[k][:, [w]]
                p = compare_peaks(r, np.abs(z), pa, ps, compute, n_lo=w * f0, label=f"c3/{name}/{compute}/w{w}",
                                  eps_series=s["max_abs"])
                peaks["max_abs_peak"] = max(peaks["max_abs_peak"], p["max_abs_peak"])
                peaks["near_ties"] += p["near_ties"]
                peaks["windows"] += p["windows"]
            # the injected template's peak stands out of the noise in its window
            wi = [w for w in wins if w in (66, 67)]
            top = max(res.peak_snr[k][tmpl[name], w] for w in wi)
            assert top > 6.0, (name, top)
            stats[name] = {**s, **peaks}
            log(f"  {name}: series {s} peaks {peaks}")
    finally:
        for h in handles:
            lloid.lloid_bank_destroy(h)
    worst = {"max_abs": max(v["max_abs"] for v in stats.values()),
             "max_rel_at6": max(v["max_rel_at6"] for v in stats.values()),
             "max_abs_peak": max(v["max_abs_peak"] for v in stats.values()),
             "near_ties": sum(v["near_ties"] for v in stats.values()),
             "windows": sum(v["windows"] for v in stats.values())}
    record_precision("batched_c3 banks 35, 36, 53 and the 131072-tap extreme, sampled 1 s windows", compute, **worst)
