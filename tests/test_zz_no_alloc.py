"""The allocation-free entry point lloid_filter_noalloc (static device scratch
of LLOID_NOALLOC_SCRATCH_BYTES per GPU) gives the results of lloid_filter:
bit-identical triggers and peak tables on two calls in a row, the first large
enough that its operand buffers need several chunks of the static scratch,
the second shorter with a ragged end; and an input whose buffers cannot fit
the scratch is refused with ENOMEM."""

import numpy as np
import pytest

from workloads import configs
from workloads.strain import Injection, inject

from gpu_util import ctx, log

pytestmark = pytest.mark.gpu


def _same(a, b, label):
    assert a.n_triggers == b.n_triggers, label
    for f in a.triggers.dtype.names:
        np.testing.assert_array_equal(a.triggers[f], b.triggers[f], err_msg=f"{label}: trigger field {f}")
    for k in ("peak_snr", "peak_sample", "peak_phase"):
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k), err_msg=f"{label}: {k}")


@pytest.mark.parametrize("compute", ["f16", "bf16", "f32"])
def test_noalloc_equals_filter_on_two_calls(compute):
    from paper_2410_16416_amd import lloid
    bank = configs.multirate_c1_bank()
    wl = configs.multirate_c1(seconds=200, detectors=1, n_injections=0, bank=bank)
    injs = [Injection(template=17, t0=60 * 2048 + 611, snr=12.0, phase=0.7),
            Injection(template=900, t0=150 * 2048 + 1500, snr=25.0, phase=-2.0)]
    x = inject(wl.strains[0], bank.family, injs)
    b = lloid.bank_from_svd(ctx(), bank, compute)
    try:
        # 200 s: the operand alone (200 s x 2048 x 480 columns) exceeds the static
        # scratch, so the allocation-free call runs several chunks of windows
        for n, label in ((200 * 2048, "200 s"), (40 * 2048 - 777, "40 s, ragged")):
            log(f"[noalloc] {compute} {label}")
            want = lloid.lloid_filter(b, 0, x[:n], window=(1, 1), peaks=True)
            got = lloid.lloid_filter_noalloc(b, 0, x[:n], window=(1, 1), peaks=True)
            _same(got, want, f"{compute} {label}")
            assert got.n_triggers > 0
            log(f"  {got.n_triggers} triggers identical")
            if n == 200 * 2048:
                w = injs[0].t0 // 2048
                assert got.peak_snr[17, w] > 0.85 * injs[0].snr
    finally:
        lloid.lloid_bank_destroy(b)


def test_noalloc_refuses_what_does_not_fit():
    from paper_2410_16416_amd import lloid
    bank = configs.mini_multirate_bank()
    b = lloid.bank_from_svd(ctx(), bank, "f16")
    try:
        # a host block whose staging copy alone fills the static scratch
        x = np.zeros(lloid.NOALLOC_SCRATCH_BYTES // 4, dtype=np.float32)
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_filter_noalloc(b, 0, x, window=(1, 1), trig_cap=16)
        assert ei.value.status == lloid.LLOID_ENOMEM
        # and the call after the refusal still matches lloid_filter
        wl = configs.mini_multirate(seconds=6, n_injections=1)
        want = lloid.lloid_filter(b, 0, wl.strains[0], window=(1, 4), peaks=True)
        got = lloid.lloid_filter_noalloc(b, 0, wl.strains[0], window=(1, 4), peaks=True)
        _same(got, want, "mini after ENOMEM")
    finally:
        lloid.lloid_bank_destroy(b)


@pytest.mark.parametrize("compute", ["f16", "f32"])
def test_noalloc_signal_consistency_in_chunks(compute):
    """With autocorrelations (signal consistency on), the allocation-free call
    carves the trigger listing slabs and the unit list out of the static
    scratch too: forced small chunks (the unit list reused chunk after chunk)
    give the triggers of lloid_filter bit for bit, xi2 included, on two calls
    in a row."""
    from paper_2410_16416_amd import lloid
    from workloads import bank_autocorrelation
    bank = configs.mini_multirate_bank()
    bank.autocorr = bank_autocorrelation(bank, 20)
    x = configs.mini_multirate(seconds=12, n_injections=2, bank=bank).strains[0]
    b = lloid.bank_from_svd(ctx(), bank, compute)
    try:
        lloid.lloid_ctx_set_chunk_bytes(ctx(), 400000)
        for n, label in ((x.shape[0], "12 s"), (5 * 1024 - 333, "5 s, ragged")):
            log(f"[noalloc xi2] {compute} {label}")
            want = lloid.lloid_filter(b, 0, x[:n], window=(1, 4), threshold=3.0)
            got = lloid.lloid_filter_noalloc(b, 0, x[:n], window=(1, 4), threshold=3.0)
            assert got.n_triggers == want.n_triggers, label
            for f in got.triggers.dtype.names:
                np.testing.assert_array_equal(got.triggers[f], want.triggers[f], err_msg=f"{label}: {f}")
            assert got.n_triggers > 10 and np.all(got.triggers["xi2"] > 0)
            log(f"  {got.n_triggers} triggers identical")
    finally:
        lloid.lloid_ctx_set_chunk_bytes(ctx(), 6 << 30)
        lloid.lloid_bank_destroy(b)
