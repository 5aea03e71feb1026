"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names the passage it follows and the kind of pin: brute force on
tiny inputs, a closed form, a library routine, a bound, or an invariant.
"""

import math

import numpy as np
import pytest
import scipy.signal
import scipy.special

import oracle
from workloads import BankSlice, SvdBank, configs
from workloads.strain import Injection, inject

Q = 32


# --------------------------------------------------------------- helpers

def brute_halfband():
    """g[n] from scalar math: 1/2 sinc(n/2) I0(10 sqrt(1-(n/32)^2)) / I0(10)."""
    g = {}
    for n in range(-Q, Q + 1):
        if n == 0:
            s = 1.0
        elif n % 2 == 0:
            s = 0.0                       # sin(k pi) = 0
        else:
            s = math.sin(math.pi * n / 2.0) / (math.pi * n / 2.0)
        g[n] = 0.5 * s * scipy.special.i0(10.0 * math.sqrt(1.0 - (n / Q) ** 2)) / scipy.special.i0(10.0)
    return g


def tiny_bank(rng, f0=16, n_t=2):
    """Random (non-SVD) three-slice bank: the oracle only needs the arrays."""
    specs = [(16, 0, 6, 3), (8, 6, 5, 2), (4, 16, 4, 2)]
    sl = []
    for rate, j, n, l in specs:
        sl.append(BankSlice(rate=rate, start_tap=j, n_taps=n,
                            basis=rng.standard_normal((l, n)),
                            mixing=rng.standard_normal((2 * n_t, l)),
                            singular_values=np.ones(l)))
    return SvdBank(f0=f0, n_templates=n_t, slices=sl)


def brute_lloid(bank, x):
    """The multi-rate form as explicit scalar sums over absolute indices."""
    g = brute_halfband()
    lo, hi = -300, 300
    T = len(x)
    levels = {0: {n: (x[n] if 0 <= n < T else 0.0) for n in range(lo, hi)}}
    n_lev = 1 + max(int(math.log2(bank.f0 // s.rate)) for s in bank.slices)
    for k in range(1, n_lev):
        prev = levels[k - 1]
        levels[k] = {m: sum(g[n] * prev.get(2 * m - n, 0.0) for n in range(-Q, Q + 1))
                     for m in range(lo, hi)}
    rows = 2 * bank.n_templates
    y = {k: {r: {n: 0.0 for n in range(lo, hi)} for r in range(rows)} for k in range(n_lev)}
    for s in bank.slices:
        d = bank.f0 // s.rate
        k = int(math.log2(d))
        for n in range(lo, hi):
            o = [sum(s.basis[l, m] * levels[k].get(n - s.start_tap // d - m, 0.0)
                     for m in range(s.n_taps)) for l in range(s.basis.shape[0])]
            for r in range(rows):
                y[k][r][n] += sum(s.mixing[r, l] * o[l] for l in range(len(o)))
    w = y[n_lev - 1]
    for k in range(n_lev - 2, -1, -1):
        nw = {}
        for r in range(rows):
            nw[r] = {}
            for n in range(lo, hi):
                acc = y[k][r][n]
                for kk in range(lo, hi):
                    dn = n - 2 * kk
                    if -Q <= dn <= Q:
                        acc += w[r][kk] * 2.0 * g[dn]
                nw[r][n] = acc
        w = nw
    out = np.array([[w[r][n] for n in range(T)] for r in range(rows)])
    return out[0::2] + 1j * out[1::2]


# ------------------------------------------------------------ resampler pins

def test_halfband_taps_match_scalar_formula_and_scipy_kaiser():
    """Resampler reading: g = 1/2 sinc(n/2) x Kaiser(beta=10), |n| <= 32."""
    g = oracle.halfband_taps()
    bg = brute_halfband()
    assert np.allclose(g, [bg[n] for n in range(-Q, Q + 1)], rtol=0, atol=1e-15)
    kais = scipy.signal.windows.kaiser(2 * Q + 1, 10.0, sym=True)
    assert np.allclose(g, 0.5 * np.sinc(np.arange(-Q, Q + 1) / 2.0) * kais, atol=1e-15)
    # half-band structure: even taps vanish except the centre, which is 1/2
    assert g[Q] == 0.5
    assert np.all(g[Q + 2::2] == 0.0) and np.all(g[:Q:2] == 0.0)
    assert abs(g.sum() - 1.0) < 1e-4            # DC gain of the decimator
    assert np.allclose(g, g[::-1])              # zero phase


def test_decimate_and_interpolate_equal_upfirdn():
    """Library pin: both resampler stages equal scipy.signal.upfirdn with the same taps."""
    rng = np.random.default_rng(1)
    g = oracle.halfband_taps()
    u = rng.standard_normal(301)
    for start in (0, 7, -5):
        d = oracle.decimate2(oracle.Seq(u, start))
        # upfirdn(h, u, up=1, down=2)[i] = sum_t h[t] u[2i - t]: absolute 2k = start - Q + 2i
        ref = scipy.signal.upfirdn(g, u, up=1, down=1)
        full_pos = start - Q + np.arange(ref.shape[0])
        ev = full_pos % 2 == 0
        assert d.start == full_pos[ev][0] // 2
        assert np.allclose(d.values, ref[ev], atol=1e-14)
        v = oracle.interpolate2(oracle.Seq(u, start))
        ref = scipy.signal.upfirdn(2.0 * g, u, up=2, down=1)
        assert v.start == 2 * start - Q
        assert np.allclose(v.values[: ref.shape[0]], ref, atol=1e-13)


def test_interpolator_passes_even_samples_exactly():
    """2g[2k] = delta_k, so v[2k] = w[k]."""
    rng = np.random.default_rng(2)
    w = oracle.Seq(rng.standard_normal(200), 11)
    v = oracle.interpolate2(w)
    assert np.allclose(v.window(22, 22 + 400)[0::2], w.values, atol=1e-14)


def test_resampler_passband_and_stopband():
    """A tone well inside the pass band survives decimate+interpolate; one past
    the band edge is suppressed (the half-band design goal)."""
    n = np.arange(4096)
    low = np.cos(2 * np.pi * 0.05 * n)
    high = np.cos(2 * np.pi * 0.45 * n)
    for tone, keep in ((low, True), (high, False)):
        d = oracle.decimate2(oracle.Seq(tone, 0))
        v = oracle.interpolate2(d).window(0, 4096)
        mid = slice(512, 3584)
        if keep:
            assert np.max(np.abs(v[mid] - tone[mid])) < 1e-3
        else:
            assert np.max(np.abs(v[mid])) < 1e-3


# ----------------------------------------------------------- brute force (P1)

def test_multirate_matches_brute_force_tiny():
    """The whole SVD multi-rate form (decimate, FIR, mix, interpolate-add)
    against explicit scalar sums on a tiny three-level bank."""
    rng = np.random.default_rng(3)
    bank = tiny_bank(rng)
    x = rng.standard_normal(32)
    z = oracle.lloid_snr(bank, x, 0, 32)
    zb = brute_lloid(bank, x)
    assert np.allclose(z, zb, rtol=1e-12, atol=1e-12)


def test_direct_form_matches_brute_force():
    rng = np.random.default_rng(4)
    h = rng.standard_normal((4, 9))
    x = rng.standard_normal(40)
    z = oracle.direct_snr(h, x, 0, 40)
    rho = np.array([[sum(h[r, j] * (x[n - j] if 0 <= n - j < 40 else 0.0) for j in range(9))
                     for n in range(40)] for r in range(4)])
    assert np.allclose(z, rho[0::2] + 1j * rho[1::2], atol=1e-13)


def test_subrange_evaluation_is_chunk_invariant():
    """P8: evaluating outputs [a, b) alone equals the same slice of a full run."""
    wl = configs.mini_multirate(seconds=8, n_injections=1)
    x = wl.strains[0]
    full = oracle.lloid_snr(wl.bank, x, 0, len(x))
    for a, b in ((0, 333), (1000, 1777), (len(x) - 500, len(x))):
        part = oracle.lloid_snr(wl.bank, x, a, b)
        assert np.allclose(part, full[:, a:b], atol=1e-12)
    sub = oracle.lloid_snr(wl.bank, x, 2000, 2600, templates=np.array([3, 7]))
    assert np.allclose(sub, full[[3, 7], 2000:2600], atol=1e-12)


def test_shift_equivariance_by_lowest_rate_period():
    """P9: delaying x by a multiple of the largest decimation delays z by the same."""
    wl = configs.mini_multirate(seconds=8, n_injections=1)
    x = wl.strains[0]
    shift = 16 * 5                               # lowest rate is f0/16
    xs = np.concatenate([np.zeros(shift), x])
    z0 = oracle.lloid_snr(wl.bank, x, 0, len(x))
    z1 = oracle.lloid_snr(wl.bank, xs, 0, len(xs))
    assert np.allclose(z1[:, shift:], z0, atol=1e-12)
    # a shift that is not a multiple of 16 changes the decimation phase
    xs3 = np.concatenate([np.zeros(3), x])
    z3 = oracle.lloid_snr(wl.bank, xs3, 0, len(xs3))
    assert not np.allclose(z3[:, 3:], z0, atol=1e-6)


# --------------------------------------------------- closed forms (P2, P3, P4)

def test_noise_free_direct_injection_peaks_at_amplitude():
    """P2: x[t0 - j] = A h_r[j] gives rho_r[t0] = A ||h_r||^2 = A, the maximum."""
    bank = configs.plain_c0_bank()
    fam = bank.family
    h = fam.full_rate_filters()
    r, a, t0 = 17, 7.5, 2000
    x = np.zeros(4096)
    x[t0 - np.arange(h.shape[1])] = a * h[r]
    z = oracle.direct_snr(h, x)
    rho = z.real if r % 2 == 0 else z.imag
    assert abs(rho[r // 2, t0] - a) < 1e-12
    assert int(np.argmax(np.abs(rho[r // 2]))) == t0


def test_single_rate_svd_recovers_projected_snr():
    """P3: for a single-rate bank, injecting filter r noise-free gives
    rho_hat_r[t0] = A sum_l M_rl^2 = A (1 - ||h_r - P h_r||^2)."""
    bank = configs.plain_c0_bank()
    sl = bank.slices[0]
    h = bank.family.full_rate_filters(n_taps=sl.n_taps)
    a, t0 = 10.0, 3000
    for r in (0, 1, 40, 127):
        x = np.zeros(6000)
        x[t0 - np.arange(sl.n_taps)] = a * h[r]
        y = oracle.lloid_snr(bank, x, t0, t0 + 1, return_real=True)
        proj = sl.basis.T @ (sl.basis @ h[r])
        loss = float(np.sum((h[r] - proj) ** 2))
        assert abs(y[r, 0] - a * (1.0 - loss)) < 1e-10
        assert abs(y[r, 0] - a * float(np.sum(sl.mixing[r] ** 2))) < 1e-10


def test_eckart_young_and_per_sample_bound():
    """P4: sum_r ||h_r - M_r U||^2 equals the discarded sigma^2, and per
    sample |rho_hat - rho| <= ||h_r - h_hat_r|| * ||x window|| (Cauchy-Schwarz)."""
    wl = configs.plain_c0(seconds=4)
    bank, x = wl.bank, wl.strains[0]
    sl = bank.slices[0]
    h = bank.family.full_rate_filters(n_taps=sl.n_taps)
    hhat = sl.mixing @ sl.basis
    resid = np.sum((h - hhat) ** 2, axis=1)
    assert abs(resid.sum() - np.sum(sl.singular_values[sl.n_basis:] ** 2)) < 1e-9
    z_svd = oracle.lloid_snr(bank, x)
    z_dir = oracle.direct_snr(h, x)
    xw = np.sqrt(np.convolve(x ** 2, np.ones(sl.n_taps))[: len(x)])   # ||x[n-N+1..n]||
    for part, rows in ((np.real, slice(0, None, 2)), (np.imag, slice(1, None, 2))):
        err = np.abs(part(z_svd) - part(z_dir))
        bound = np.sqrt(resid[rows])[:, None] * xw[None, :]
        assert np.all(err <= bound * (1 + 1e-9) + 1e-12)
    # in white noise the mean squared error equals ||h - h_hat||^2 (statistically)
    err2 = np.mean((z_svd.real - z_dir.real)[:, sl.n_taps:] ** 2, axis=1)
    assert np.allclose(err2, resid[0::2], rtol=0.35, atol=1e-6)


def test_sigma2_equals_projected_norms_single_rate():
    """sigma2_i = ||P h_cos||^2 + ||P h_sin||^2 for a single-rate bank."""
    bank = configs.plain_c0_bank()
    sl = bank.slices[0]
    h = bank.family.full_rate_filters(n_taps=sl.n_taps)
    p = h @ sl.basis.T
    want = (p ** 2).sum(axis=1)
    assert np.allclose(oracle.sigma2(bank), want[0::2] + want[1::2], atol=1e-12)


# ------------------------------------------------------- statistics (P5, P7)

def test_noise_moments_match_sigma2_multirate():
    """P5: in unit white noise E|z_i|^2 = sigma2_i (including the 1/D_s weight
    of the low-rate slices); checked by the sample mean over a long stretch."""
    wl = configs.mini_multirate(seconds=200, n_injections=0)
    bank, x = wl.bank, wl.strains[0]
    z = oracle.lloid_snr(bank, x, 4096, len(x))
    s2 = oracle.sigma2(bank)
    m = np.mean(np.abs(z) ** 2, axis=1)
    # successive samples are correlated; allow ~5 sigma of the effective count
    assert np.allclose(m, s2, rtol=0.06)
    # dropping the 1/D weight would overestimate by far more than that
    wrong = sum(((sl.mixing ** 2).sum(1)[0::2] + (sl.mixing ** 2).sum(1)[1::2]) for sl in bank.slices)
    assert np.max(np.abs(m - wrong) / wrong) > 0.5


def _effective_filters(bank, n_taps, period, lag_lo, lag_hi):
    """Impulse-probe the multi-rate system: it is linear and periodically
    time-varying with period D_max, so Y[n] = sum_j heff[n mod D][:, j] x[n - j]."""
    base = 4 * period * 32
    T = base + period + lag_hi + 8
    rows = 2 * bank.n_templates
    heff = np.zeros((period, rows, lag_hi - lag_lo))
    js = np.arange(lag_lo, lag_hi)
    for p in range(period):
        xi = np.zeros(T)
        xi[base + p] = 1.0
        ys = oracle.lloid_snr(bank, xi, return_real=True)
        n = base + p + js
        for q in range(period):
            m = (n % period) == q
            heff[q][:, js[m] - lag_lo] = ys[:, n[m]]
    return heff


def test_full_rank_multirate_matches_direct_form():
    """P7: with full-rank slices the multi-rate form is the exact matched filter
    up to the resampler and slice-edge errors.  Those errors are a linear
    periodically time-varying filter mismatch, measured by impulse probing;
    the multi-rate output must equal the probed system exactly and stay
    within ||heff - h|| ||x|| of the direct form (Cauchy-Schwarz)."""
    fam_bank = configs.mini_multirate_bank()
    fam = fam_bank.family
    from workloads import build_svd_bank, SliceSpec
    specs = [SliceSpec(s.rate, s.start_tap, s.n_taps, s.n_taps) for s in fam_bank.slices]
    full = build_svd_bank(fam, fam_bank.f0, specs)
    inj = [Injection(template=5, t0=6000, snr=20.0, phase=0.3)]
    rng = np.random.default_rng(6)
    x = inject(0.3 * rng.standard_normal(8192), fam, inj)
    h = fam.full_rate_filters()
    zd = oracle.direct_snr(h, x)
    zs = oracle.lloid_snr(full, x)
    peak = np.abs(zd[5, 6000])
    assert peak > 19.0
    assert abs(np.abs(zs[5, 6000]) - peak) < 1e-2 * peak

    period, n_taps = 16, h.shape[1]
    lag_lo, lag_hi = -1100, n_taps + 1100
    heff = _effective_filters(full, n_taps, period, lag_lo, lag_hi)
    assert np.abs(heff[:, :, :50]).max() < 1e-14 and np.abs(heff[:, :, -50:]).max() < 1e-14
    hext = np.zeros((h.shape[0], lag_hi - lag_lo))
    hext[:, -lag_lo:-lag_lo + n_taps] = h
    mism = np.linalg.norm(heff - hext[None], axis=2)          # [phase, row]
    assert mism.max() < 0.1                                   # unit-norm filters
    xs = oracle.Seq(x, 0)
    ys = np.concatenate([zs.real[:, None], zs.imag[:, None]], axis=1).reshape(-1, zs.shape[1])
    yd = np.concatenate([zd.real[:, None], zd.imag[:, None]], axis=1).reshape(-1, zd.shape[1])
    for n in range(3000, 8192, 97):
        seg = xs.window(n - lag_hi + 1, n - lag_lo + 1)[::-1]  # seg[j - lag_lo] = x[n - j]
        q = n % period
        assert np.allclose(heff[q] @ seg, ys[:, n], atol=1e-10)
        bound = mism[q] * np.linalg.norm(seg)
        assert np.all(np.abs(ys[:, n] - yd[:, n]) <= bound + 1e-10)

    # the single-rate special case (S = 1, D = 1) is exactly the direct form at full rank
    sr = build_svd_bank(fam, fam_bank.f0, [SliceSpec(1024, 0, 4096, 32)])
    zsr = oracle.lloid_snr(sr, x)
    assert np.max(np.abs(zsr - zd)) < 1e-9


# ------------------------------------------------------ windows, peaks (P10)

def test_window_edges_c0():
    """0.1 s windows at 1024 Hz: [floor(102.4 w), floor(102.4 (w+1))) -> 102 or 103 samples."""
    st = oracle.window_starts(80, 1024, 1, 10)
    assert st[0] == 0 and st[80] == 8192
    lens = np.diff(st)
    assert set(lens.tolist()) == {102, 103}
    assert st[40] == 4096 and st[41] == 4198     # window 40 holds the C0 injection at 4146
    n = np.arange(8192)
    w = oracle.window_index(n, 1024, 1, 10)
    for k in range(80):
        assert np.all(w[st[k]:st[k + 1]] == k)


def test_peak_table_and_triggers_brute_force():
    rng = np.random.default_rng(5)
    z = (rng.standard_normal((5, 700)) + 1j * rng.standard_normal((5, 700))) * 2.5
    z[2, 100] = z[2, 101] = 9.0                  # a tie: the lower index wins
    z[3, 250] = 4.0                              # exactly at threshold: kept
    n_lo = 37
    wins, pa, ps, ph = oracle.peak_table(z, n_lo, 1024, 1, 10)
    trig = oracle.triggers(z, n_lo, 1024, 1, 10, threshold=4.0)
    st = oracle.window_starts(20, 1024, 1, 10)
    want = []
    for r in range(5):
        for c, w in enumerate(wins):
            best, arg = -1.0, -1
            for n in range(max(st[w], n_lo), min(st[w + 1], n_lo + 700)):
                v = abs(z[r, n - n_lo])
                if v > best:
                    best, arg = v, n
            assert abs(pa[r, c] - best) <= 1e-15 * best and ps[r, c] == arg
            zz = z[r, arg - n_lo]
            assert abs(ph[r, c] - math.atan2(zz.imag, zz.real)) < 1e-14
            if best >= 4.0:
                want.append((r, int(w), arg))
    assert [(t[0], t[1], t[2]) for t in trig] == want
    assert ps[2, list(wins).index(oracle.window_index(np.array([n_lo + 100]), 1024, 1, 10)[0])] == n_lo + 100


# ------------------------------------------------------------- end to end C0

def test_c0_injection_recovered_in_window_40():
    """The C0 workload: SNR-10 injection at sample 4146 (window 40); both forms
    find it there with |z| close to 10, the SVD form lower by its projection loss."""
    wl = configs.plain_c0()
    bank, x = wl.bank, wl.strains[0]
    inj = wl.injections[0]
    h = bank.family.full_rate_filters(n_taps=1024)
    zd = oracle.direct_snr(h, x)
    zs = oracle.lloid_snr(bank, x)
    for z in (zd, zs):
        wins, pa, ps, _ = oracle.peak_table(z, 0, 1024, 1, 10)
        assert pa.shape == (64, 80)
        assert ps[inj.template, 40] == 4146
        assert 8.0 < pa[inj.template, 40] < 12.0
    assert abs(np.abs(zs[inj.template, 4146]) - np.abs(zd[inj.template, 4146])) < 0.2


def test_subsample_peak_recovers_a_sampled_parabola():
    """Closed form: three samples of c - k (t - t0)^2 give back t0 and c."""
    rng = np.random.default_rng(4)
    t0 = rng.uniform(-0.49, 0.49, 200)
    c = rng.uniform(4.0, 30.0, 200)
    k = rng.uniform(0.01, 3.0, 200)

    def a(t):
        return c - k * (t - t0) ** 2

    dt, v = oracle.subsample_peak(a(-1.0), a(0.0), a(1.0))
    assert np.allclose(dt, t0, rtol=0, atol=1e-12)
    assert np.allclose(v, c, rtol=0, atol=1e-12)


def test_subsample_peak_degenerate_and_clipped_cases():
    # flat and convex triples keep the sampled value
    assert oracle.subsample_peak(5.0, 5.0, 5.0) == (0.0, 5.0)
    assert oracle.subsample_peak(6.0, 5.0, 6.0) == (0.0, 5.0)
    # a vertex beyond the bracket is clipped to half a sample
    dt, v = oracle.subsample_peak(1.0, 5.0, 6.0)
    assert dt == 0.5 and v == pytest.approx(5.0 + 0.25 * 5.0 * 0.5, abs=1e-15)
    # symmetric neighbours: the sample is the peak
    dt, v = oracle.subsample_peak(3.0, 7.0, 3.0)
    assert dt == 0.0 and v == 7.0


def test_subsample_peak_recovers_a_fractional_arrival():
    """A noise-free chirp arriving between samples (band-limited fractional
    delay by an FFT phase ramp): the exact matched filter's sampled peak is
    low by the sampling loss; the parabola brings back the arrival time and
    most of the lost SNR."""
    from workloads.chirp import mass_chirps
    f0, n, t_c, amp = 1024, 8192, 5000, 10.0
    fam = mass_chirps(1, f0, 1.0, 20.0, 1.2, 1.2, np.random.default_rng(0))
    h = fam.full_rate_filters()                        # [2, 1024] cos, sin; unit norm
    x = np.zeros(n)
    j = np.arange(h.shape[1])
    x[t_c - j] = amp * h[0]                            # the cos filter, coalescing at t_c
    f = np.fft.rfftfreq(n)
    for tau in (0.25, 0.5, -0.4):
        xs = np.fft.irfft(np.fft.rfft(x) * np.exp(-2j * np.pi * f * tau), n)
        a = np.abs(oracle.direct_snr(h, xs, 0, n)[0])
        k = int(np.argmax(a))
        dt, v = oracle.subsample_peak(a[k - 1], a[k], a[k + 1])
        peak_true = np.abs(oracle.direct_snr(h, x, t_c, t_c + 1)[0, 0])   # the aligned peak
        assert abs((k + dt) - (t_c + tau)) < 0.05, tau
        assert abs(v - peak_true) < 0.35 * abs(a[k] - peak_true), tau


# ------------------------------------------------- signal consistency (xi^2)

def _rand_acorr(rng, half):
    """A Hermitian lag table with R[0] = 1 and |R| < 1 elsewhere."""
    r = np.zeros(2 * half + 1, dtype=np.complex128)
    r[half] = 1.0
    for k in range(1, half + 1):
        v = 0.8 ** k * np.exp(1j * rng.uniform(0, 2 * np.pi))
        r[half + k] = v
        r[half - k] = np.conj(v)
    return r


def test_autocorrelation_input_matches_numpy_correlate():
    """The bank's lag table (setup stage) against the library correlation:
    np.correlate(h, h, 'full')[N - 1 + k] = sum_j h[j] conj(h[j - k])."""
    from workloads import autocorrelation
    rng = np.random.default_rng(11)
    f = rng.standard_normal((6, 29))
    r = autocorrelation(f, 7)
    for i in range(3):
        h = f[2 * i] + 1j * f[2 * i + 1]
        c = np.correlate(h, h, "full") / np.sum(np.abs(h) ** 2)
        assert np.allclose(r[i], c[28 - 7:28 + 8], atol=1e-14)
        assert abs(r[i, 7] - 1.0) < 1e-14
        assert np.allclose(r[i, ::-1], np.conj(r[i]), atol=1e-14)


def test_xi2_vanishes_on_a_pure_template_response_and_counts_a_defect():
    """Closed form: if z[n* + k] = c R[k] on every lag, each numerator term is
    zero; adding e at one in-range lag k0 != 0 gives |e|^2 / sum (2 - 2|R|^2);
    a defect outside the lag range, or outside [0, n_end), changes nothing.
    A transposed lag (R[-k]) or a missing conjugate fails the first case."""
    rng = np.random.default_rng(12)
    half = 5
    r = _rand_acorr(rng, half)
    c = 7.0 * np.exp(0.7j)
    n_star, n_lo = 40, 30
    z = np.zeros(30, dtype=np.complex128)
    z[n_star - half - n_lo:n_star + half + 1 - n_lo] = c * r
    den = np.sum(2.0 - 2.0 * np.abs(r) ** 2)
    assert oracle.xi2(z, n_lo, 1000, n_star, r) < 1e-24
    z2 = z.copy()
    e = 0.3 - 0.2j
    z2[n_star + 3 - n_lo] += e
    assert abs(oracle.xi2(z2, n_lo, 1000, n_star, r) - abs(e) ** 2 / den) < 1e-14
    z3 = z.copy()
    z3[n_star + half + 2 - n_lo] += 5.0                  # beyond the lag range
    assert oracle.xi2(z3, n_lo, 1000, n_star, r) < 1e-24
    # the series ends at n_end = n* + 2: lags 3..5 drop out of both sums
    den_c = np.sum(2.0 - 2.0 * np.abs(r[:half + 3]) ** 2)
    assert abs(oracle.xi2(z2, n_lo, n_star + 3, n_star, r) - 0.0) < 1e-24
    z4 = z.copy()
    z4[n_star - 2 - n_lo] += e
    assert abs(oracle.xi2(z4, n_lo, n_star + 3, n_star, r) - abs(e) ** 2 / den_c) < 1e-14
    # the start of the data clips the negative lags the same way
    z5 = np.zeros(12, dtype=np.complex128)
    z5[:1 + half] = c * r[half - 0:]
    z5[1] += e
    den_s = np.sum(2.0 - 2.0 * np.abs(r[half:]) ** 2)
    assert abs(oracle.xi2(z5, 0, 1000, 0, r) - abs(e) ** 2 / den_s) < 1e-14
    # a transposed lag table is caught by the pure response
    assert oracle.xi2(z, n_lo, 1000, n_star, r[::-1]) > 1e-3


def test_xi2_averages_one_in_white_noise():
    """Closed-form expectation: with z the exact matched filter of unit-norm
    cos/sin filters in unit white noise and R their autocorrelation,
    E|z[n+k] - z[n] R[k]|^2 = 2 - 2|R[k]|^2 at any fixed n, so xi2 averages 1
    (Sec. II.A's consistency value, normalised as restated in the oracle).
    Dropping the conjugate in the lag table gives 2 + 2|R|^2 - 4 Re R^2
    instead, caught below."""
    from workloads import autocorrelation
    from workloads.chirp import mass_chirps
    f0, n = 1024, 1 << 17
    fam = mass_chirps(2, f0, 0.5, 20.0, 1.2, 2.0, np.random.default_rng(3))
    h = fam.full_rate_filters()
    half = 24
    r = autocorrelation(h, half)
    x = np.random.default_rng(4).standard_normal(n)
    z = oracle.direct_snr(h, x, 0, n)
    pos = np.arange(2000, n - 2000, 37)
    for i in range(2):
        v = np.array([oracle.xi2(z[i], 0, n, int(p), r[i]) for p in pos])
        # neighbouring positions are nearly independent at this spacing
        se = np.std(v) / np.sqrt(len(v))
        assert abs(np.mean(v) - 1.0) < 5 * se + 0.01, (i, np.mean(v), se)
        w = np.array([oracle.xi2(z[i], 0, n, int(p), np.conj(r[i])) for p in pos[:400]])
        assert np.max(np.abs(r[i].imag)) > 0.3 and np.mean(w) > 1.5


# --------------------------------------------------- coincidence (Sec. II.A)

def _trig(rows):
    from workloads.triggers import TRIGGER_DTYPE
    t = np.zeros(len(rows), dtype=TRIGGER_DTYPE)
    for k, (bank, tmpl, sample, snr, dt) in enumerate(rows):
        t[k]["bank"], t[k]["template_id"], t[k]["sample"] = bank, tmpl, sample
        t[k]["snr"], t[k]["dt"] = snr, dt
    return t


def test_coincidence_hand_example():
    """Worked by hand: same bank and template within 10 samples (inclusive)."""
    a = _trig([(0, 5, 100, 6.0, 0.25), (0, 5, 2000, 5.0, 0.0), (0, 6, 100, 4.0, 0.0)])
    b = _trig([(0, 5, 90, 8.0, -0.25), (0, 5, 111, 4.5, 0.0), (0, 6, 300, 4.0, 0.0), (1, 5, 100, 9.0, 0.0)])
    pairs, bg = oracle.coincidences(a, b, 10)
    assert [(p[0], p[1]) for p in pairs] == [(0, 0)]
    assert abs(pairs[0][4] - 10.0) < 1e-12            # sqrt(6^2 + 8^2)
    assert abs(pairs[0][5] - (-10.5)) < 1e-12         # (90 - 0.25) - (100 + 0.25)
    assert bg == [0, 1, 1, 0, 1, 1, 1]
    pairs11, _ = oracle.coincidences(a, b, 11)
    assert [(p[0], p[1]) for p in pairs11] == [(0, 0), (0, 1)]


def test_coincidence_invariants():
    """Swapping the detectors swaps the pairs and negates dt; shifting every
    sample by a constant changes nothing; an unbounded max_dt pairs every
    trigger with every trigger of its (bank, template) in the other list."""
    from workloads.triggers import trigger_pair
    a, b = trigger_pair(5, n_banks=2, n_templates=12, n_windows=10, rate=0.3)
    p, bg = oracle.coincidences(a, b, 25)
    q, bgq = oracle.coincidences(b, a, 25)
    assert sorted((x[1], x[0]) for x in p) == sorted((x[0], x[1]) for x in q)
    dts = {(x[0], x[1]): x[5] for x in p}
    assert all(abs(dts[(x[1], x[0])] + x[5]) < 1e-9 for x in q)
    assert bg[:len(a)] == bgq[len(b):] and bg[len(a):] == bgq[:len(b)]
    a2, b2 = a.copy(), b.copy()
    a2["sample"] += 123457
    b2["sample"] += 123457
    assert [x[:2] for x in oracle.coincidences(a2, b2, 25)[0]] == [x[:2] for x in p]
    allp, _ = oracle.coincidences(a, b, 10 ** 9)
    from collections import Counter
    ca = Counter(zip(a["bank"].tolist(), a["template_id"].tolist()))
    cb = Counter(zip(b["bank"].tolist(), b["template_id"].tolist()))
    assert len(allp) == sum(ca[k] * cb[k] for k in ca)
    assert len(p) < len(allp)


# ---------------------------------------- conditioning: PSD, whitening, gating

def test_welch_psd_equals_scipy():
    """Library routine: the block PSD is scipy's Welch average (periodic Hann,
    half overlap, no detrending, density scaling)."""
    x = np.random.default_rng(31).standard_normal(40000) * 2.5
    for L in (256, 1024):
        _, want = scipy.signal.welch(x, fs=1024, window="hann", nperseg=L, noverlap=L // 2, detrend=False,
                                     average="mean", scaling="density")
        assert np.allclose(oracle.welch_psd(x, 1024, L), want, rtol=1e-12, atol=0)


def test_whitening_with_a_flat_psd_is_a_scaling():
    """Closed form: with S = 2 sigma^2 / f0 the gain is 1/sigma on every bin and
    the half-overlapped Hann windows sum to one, so whitening returns x/sigma
    exactly (a dropped segment, a wrong hop or window fails it); scaling the
    PSD by c scales the output by 1/sqrt(c)."""
    rng = np.random.default_rng(32)
    x = rng.standard_normal(5000 + 77)
    for L in (256, 512):
        flat = np.full(L // 2 + 1, 2.0 * 9.0 / 1024)
        assert np.allclose(oracle.whiten(x, 1024, L, flat), x / 3.0, atol=1e-12)
        s = oracle.welch_psd(x, 1024, L)
        assert np.allclose(oracle.whiten(x, 1024, L, 4.0 * s), oracle.whiten(x, 1024, L, s) / 2.0, atol=1e-12)


def test_whitening_flattens_coloured_noise():
    """AR(1) noise y[n] = a y[n-1] + e[n] has the one-sided density
    S(f) = (2/f0) / |1 - a e^{-2 pi i f/f0}|^2; whitened with it (or with the
    block's own estimate), the output has unit variance and a flat PSD."""
    f0, L, a = 1024, 512, 0.9
    e = np.random.default_rng(33).standard_normal(1 << 18)
    y = scipy.signal.lfilter([1.0], [1.0, -a], e)
    f = np.arange(L // 2 + 1) / L
    true = (2.0 / f0) / np.abs(1.0 - a * np.exp(-2j * np.pi * f)) ** 2
    for s in (true, oracle.welch_psd(y, f0, L)):
        xw = oracle.whiten(y, f0, L, s)[L:-L]
        assert abs(np.var(xw) - 1.0) < 0.03
        flat = oracle.welch_psd(xw, f0, L)[4:-4] * f0 / 2.0
        assert np.all(np.abs(flat - 1.0) < 0.2)
    assert np.var(y) > 4.0     # the input was far from white


def test_gate_zeroes_around_loud_samples():
    """Closed form: a spike above the threshold zeroes exactly 2G+1 samples
    around it (clipped at the ends of the data); the rest is unchanged."""
    rng = np.random.default_rng(34)
    xw = rng.standard_normal(3000)
    xw[1000] = 80.0
    xw[5] = -90.0
    out, n = oracle.gate(xw, 20.0, 50)
    assert n == 101 + 56
    assert np.all(out[950:1051] == 0) and np.all(out[:56] == 0)
    keep = np.ones(3000, bool)
    keep[950:1051] = False
    keep[:56] = False
    assert np.array_equal(out[keep], xw[keep])
    assert oracle.gate(xw, 0.0, 50)[1] == 0
