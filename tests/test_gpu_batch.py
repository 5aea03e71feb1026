"""Batched filtering: many uneven banks in one launch per stage.

Each bank's peaks and triggers in a batch must equal those of the bank alone,
bit for bit (every output is accumulated in the same order whatever the tile,
chunk or batch it lands in), and must match the FP64 oracle.
"""

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


@pytest.mark.parametrize("compute", ["f16", "f32"])
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
            for fv in range(3):
                for mv in range(4):
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
        for mv in range(4):
            lloid.lloid_ctx_set_tiles(c, 0, mv)
            r = lloid.lloid_filter(handles[0], 0, x, window=(3, 4), threshold=3.0,
                                   snr_out=np.zeros((banks[0].n_templates, x.size, 2), np.float32))
            if series is None:
                series = r.snr
            else:
                assert np.array_equal(r.snr, series), mv
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_ctx_set_tiles(c, 3, 0)
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
        assert res.shape[0] == 3 * 4 and np.all(res["ms"] > 0)   # FIR x mixing shapes
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
