"""Coincidence of two detectors' triggers on the device (Sec. II.A, the
coincidence generator): every pair, its network SNR and arrival difference,
and the background flags must equal the oracle's definition on seeded
synthetic trigger lists; the error paths, and the injections of a
two-detector filter run found as coincidences."""

import numpy as np
import pytest

import oracle
from workloads import configs
from workloads.triggers import trigger_pair

from gpu_util import ctx, log

pytestmark = pytest.mark.gpu


def _check(got, bg, a, b, max_dt):
    pairs, want_bg = oracle.coincidences(a, b, max_dt)
    assert got.shape[0] == len(pairs)
    if pairs:
        w = np.array([(p[0], p[1], p[2], p[3]) for p in pairs], dtype=np.int64)
        assert np.array_equal(got["a"], w[:, 0]) and np.array_equal(got["b"], w[:, 1])
        assert np.array_equal(got["bank"], w[:, 2]) and np.array_equal(got["template_id"], w[:, 3])
        snr = np.array([p[4] for p in pairs])
        dt = np.array([p[5] for p in pairs])
        # FP32 sums of FP32 inputs: a few ulps of the operands
        assert np.all(np.abs(got["snr_net"] - snr) <= 1e-6 * snr)
        assert np.all(np.abs(got["dt"] - dt) <= 1e-6 * (np.abs(dt) + 1.0))
    assert bg.tolist() == want_bg
    return len(pairs)


@pytest.mark.parametrize("seed,max_dt", [(1, 0), (2, 21), (3, 200), (4, 5000)])
def test_coincide_matches_oracle(seed, max_dt):
    from paper_2410_16416_amd import lloid
    a, b = trigger_pair(seed)
    log(f"[coinc] seed={seed} max_dt={max_dt} n_a={len(a)} n_b={len(b)}")
    got, bg = lloid.lloid_coincide(ctx(), a, b, max_dt, background=True)
    n = _check(got, bg, a, b, max_dt)
    log(f"  {n} pairs, {int(bg.sum())} background")


def test_coincide_device_lists_and_capacity():
    """Device-resident lists give the host result; a capacity below the pair
    count returns ETRUNC with the count needed; the binding then retries."""
    import ctypes
    import torch
    from paper_2410_16416_amd import lloid
    a, b = trigger_pair(7)
    host = lloid.lloid_coincide(ctx(), a, b, 30)
    da = torch.from_numpy(a.view(np.uint8).copy()).to("cuda")
    db = torch.from_numpy(b.view(np.uint8).copy()).to("cuda")
    dev = lloid.lloid_coincide(ctx(), da, db, 30)
    assert np.array_equal(host, dev) and host.shape[0] > 10
    out = np.zeros(4, dtype=lloid.COINC_DTYPE)
    n = ctypes.c_int64(0)
    st = lloid._lib.lloid_coincide(ctx(), a.ctypes.data, len(a), b.ctypes.data, len(b), 30, out.ctypes.data, 4,
                                   ctypes.byref(n), None)
    assert st == lloid.LLOID_ETRUNC and n.value == host.shape[0]
    assert np.array_equal(out, host[:4])


def test_coincide_edge_cases():
    from paper_2410_16416_amd import lloid
    a, b = trigger_pair(8, n_banks=1, n_templates=5, n_windows=6, rate=0.5)
    empty = a[:0]
    got, bg = lloid.lloid_coincide(ctx(), empty, b, 10, background=True)
    assert got.shape[0] == 0 and bg.tolist() == [1] * len(b)
    got, bg = lloid.lloid_coincide(ctx(), a, empty, 10, background=True)
    assert got.shape[0] == 0 and bg.tolist() == [1] * len(a)
    got = lloid.lloid_coincide(ctx(), empty, empty, 10)
    assert got.shape[0] == 0
    # one key only, every pair within reach
    one_a = a[(a["bank"] == 0) & (a["template_id"] == 0)]
    one_b = b[(b["bank"] == 0) & (b["template_id"] == 0)]
    got, bg = lloid.lloid_coincide(ctx(), one_a, one_b, 10 ** 9, background=True)
    _check(got, bg, one_a, one_b, 10 ** 9)
    assert got.shape[0] == len(one_a) * len(one_b)
    # a list out of order, a negative max_dt
    bad = a[::-1].copy()
    with pytest.raises(lloid.LloidError) as ei:
        lloid.lloid_coincide(ctx(), bad, b, 10)
    assert ei.value.status == lloid.LLOID_EINVAL
    with pytest.raises(lloid.LloidError) as ei:
        lloid.lloid_coincide(ctx(), b, bad, 10)
    assert ei.value.status == lloid.LLOID_EINVAL
    with pytest.raises(lloid.LloidError) as ei:
        lloid.lloid_coincide(ctx(), a, b, -1)
    assert ei.value.status == lloid.LLOID_EINVAL


def test_injections_are_coincident_across_detectors():
    """Two detectors with the same injections: each injection's template has a
    coincidence at the injection time, with a network SNR near sqrt(2) times
    the injected SNR (the bank's SVD loss and the noise aside)."""
    from paper_2410_16416_amd import lloid
    wl = configs.mini_multirate(seconds=12, detectors=2, n_injections=2)
    h = lloid.bank_from_svd(ctx(), wl.bank, "f16")
    try:
        trig = [lloid.lloid_filter(h, d, x, window=(1, 4)).triggers for d, x in enumerate(wl.strains)]
    finally:
        lloid.lloid_bank_destroy(h)
    max_dt = 11   # 10 ms at 1024 Hz, rounded up
    got = lloid.lloid_coincide(ctx(), trig[0], trig[1], max_dt)
    log(f"[coinc e2e] {len(trig[0])} + {len(trig[1])} triggers, {got.shape[0]} coincidences")
    for inj in wl.injections:
        hit = got[(got["template_id"] == inj.template)]
        samples = trig[0]["sample"][hit["a"]]
        near = np.abs(samples - inj.t0) <= 2
        assert near.any(), inj
        best = float(hit["snr_net"][near].max())
        assert abs(best - np.sqrt(2.0) * inj.snr) < 0.25 * inj.snr, (best, inj.snr)
