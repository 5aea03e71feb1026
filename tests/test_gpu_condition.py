"""Conditioning before the filter on the device (Sec. II.A: PSD, whitening
with it, gating of large whitened deviations), against the FP64 oracle.

Tolerance: the device runs a radix-2 FFT in FP32 on FP32 strain; its error
relative to a segment's RMS is of order eps32 * log2(L) (~1e-6 here), and
the PSD is a mean of FP32 periodograms summed in FP64 (relative error of
order eps32); 1e-4 of the output's unit RMS (absolute) and 1e-5 relative on
the PSD leave margin.  Gate decisions are compared where no whitened sample
lies near the threshold (planted glitches far above it, noise far below).
"""

import numpy as np
import pytest
import scipy.signal

import oracle
from workloads import configs

from gpu_util import ctx, log

pytestmark = pytest.mark.gpu

F0 = 1024


def _ar1(n, a, seed, scale=1.0):
    e = np.random.default_rng(seed).standard_normal(n)
    return scale * scipy.signal.lfilter([1.0], [1.0, -a], e)


@pytest.mark.parametrize("L,a", [(256, 0.0), (1024, 0.9), (4096, 0.5)])
def test_condition_matches_oracle(L, a):
    from paper_2410_16416_amd import lloid
    x = _ar1(40000 + 77, a, 41 + L, scale=2.5)
    out, psd, gated = lloid.lloid_condition(ctx(), F0, x, L)
    want_psd = oracle.welch_psd(x, F0, L)
    want = oracle.whiten(x, F0, L, want_psd)
    log(f"[condition] L={L} a={a}: max |d out| {np.max(np.abs(out - want)):.2e}, "
        f"max rel d psd {np.max(np.abs(psd - want_psd) / want_psd):.2e}")
    assert gated == 0
    assert np.allclose(psd, want_psd, rtol=1e-5, atol=0)
    assert np.max(np.abs(out - want)) < 1e-4
    assert abs(np.std(out[L:-L]) - 1.0) < 0.05


def test_condition_with_given_psd_and_device_buffers():
    import torch
    from paper_2410_16416_amd import lloid
    L, a = 512, 0.9
    x = _ar1(30000, a, 43)
    f = np.arange(L // 2 + 1) / L
    true = (2.0 / F0) / np.abs(1.0 - a * np.exp(-2j * np.pi * f)) ** 2
    out, psd, _ = lloid.lloid_condition(ctx(), F0, x, L, psd=true)
    # the device applies a caller's PSD rounded to FP32 and reports that
    assert np.array_equal(psd, true.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(out - oracle.whiten(x, F0, L, true))) < 1e-4
    dx = torch.from_numpy(x).to("cuda")
    dout = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
    lloid.lloid_condition(ctx(), F0, dx, L, psd=true, out=dout)
    assert np.array_equal(dout.cpu().numpy(), out)


def test_gating_matches_oracle():
    from paper_2410_16416_amd import lloid
    L, G, thr = 1024, 100, 20.0
    x = np.random.default_rng(44).standard_normal(50000) * 3.0
    for n0, amp in ((5000, 3000.0), (30000, -2500.0), (49990, 4000.0), (20, 3500.0)):
        x[n0] += amp
    out, psd, gated = lloid.lloid_condition(ctx(), F0, x, L, gate_threshold=thr, gate_half_width=G)
    s, want, want_gated = oracle.condition(x, F0, L, thr, G)
    xw = oracle.whiten(x, F0, L, s)
    margin = np.abs(np.abs(xw) - thr)
    assert margin.min() > 1.0          # no whitened sample near the threshold
    log(f"[gate] {gated} samples gated (oracle {want_gated})")
    assert gated == want_gated > 0
    assert np.array_equal(out == 0, want == 0)
    assert np.max(np.abs(out - want)) < 1e-4


def test_condition_errors():
    from paper_2410_16416_amd import lloid
    x = np.random.default_rng(45).standard_normal(3000)
    for L in (3000, 32, 8192):
        with pytest.raises(lloid.LloidError) as ei:
            lloid.lloid_condition(ctx(), F0, x, L)
        assert ei.value.status == lloid.LLOID_EINVAL
    with pytest.raises(lloid.LloidError) as ei:
        lloid.lloid_condition(ctx(), F0, x[:200], 256)       # shorter than a segment, no PSD
    assert ei.value.status == lloid.LLOID_EINVAL
    out, _, _ = lloid.lloid_condition(ctx(), F0, x[:200], 256, psd=np.full(129, 2.0 / F0))
    assert np.allclose(out, x[:200], atol=1e-5)               # flat unit PSD: the identity
    bad = x.copy()
    bad[10] = np.nan
    with pytest.raises(lloid.LloidError) as ei:
        lloid.lloid_condition(ctx(), F0, bad, 256)
    assert ei.value.status == lloid.LLOID_EDATA


def test_conditioned_strain_feeds_the_filter():
    """White noise of variance 9 with injections scaled by 3 and a loud
    glitch: whitened with the PSD of the first 4 s (before the glitch, which
    would dominate a mean PSD over the block) and gated, the strain gives the
    filter the injections near their SNRs, and the glitch, which alone makes
    triggers in many templates, leaves none."""
    from paper_2410_16416_amd import lloid
    wl = configs.mini_multirate(seconds=12, n_injections=2)
    x = 3.0 * wl.strains[0]
    g0 = 9000
    x[g0] += 4000.0
    h = lloid.bank_from_svd(ctx(), wl.bank, "f16")
    try:
        raw = lloid.lloid_filter(h, 0, x / 3.0, window=(1, 4)).triggers
        _, psd0, _ = lloid.lloid_condition(ctx(), F0, x[:4096], 512)
        cond, _, gated = lloid.lloid_condition(ctx(), F0, x, 512, gate_threshold=25.0, gate_half_width=256,
                                               psd=psd0)
        res = lloid.lloid_filter(h, 0, cond.astype(np.float64), window=(1, 4)).triggers
    finally:
        lloid.lloid_bank_destroy(h)
    assert all(abs(inj.t0 - g0) > 1024 for inj in wl.injections)
    glitch_w = g0 // 256
    log(f"[condition e2e] gated {gated}; triggers near the glitch raw "
        f"{int(np.sum(np.abs(raw['window'] - glitch_w) <= 1))}, conditioned {int(np.sum(np.abs(res['window'] - glitch_w) <= 1))}")
    assert gated >= 513
    assert np.sum(np.abs(raw["window"] - glitch_w) <= 1) > 5
    assert np.sum((np.abs(res["window"] - glitch_w) <= 1) & (res["snr"] > 6)) == 0
    for inj in wl.injections:
        hit = res[(res["template_id"] == inj.template) & (np.abs(res["sample"] - inj.t0) <= 2)]
        assert hit.shape[0] == 1 and abs(float(hit["snr"][0]) - inj.snr) < 0.15 * inj.snr, (inj, hit)
