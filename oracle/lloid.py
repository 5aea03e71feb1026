"""Plain FP64 statement of the LLOID filtering path (test infrastructure only).

The paper states the method in Sec. II.A: the conditioned data are
down-sampled, cross-correlated with the orthogonal (basis) templates of each
time slice, the orthogonal SNR series are multiplied by the SVD
coefficients, and the physical SNR segments are up-sampled and summed; SNR
peaks of at least 4 become triggers (Fig. 1 caption, Sec. II.A, Table I
caption).  Everything it leaves open is fixed here as follows:

* Sequences live on all integers; full-rate strain x[n] is zero outside
  [0, T).  A ``Seq`` holds the values on [start, start + len) and is zero
  elsewhere, so every finite filter below is evaluated exactly.
* Resampling uses one zero-phase half-band filter,
      g[n] = 1/2 sinc(n/2) I0(beta sqrt(1 - (n/Q)^2)) / I0(beta),  |n| <= Q,
  with Q = 32, beta = 10, aligned to absolute sample 0:
      decimate:    d[k] = sum_n g[n] u[2k - n]
      interpolate: v[n] = sum_k w[k] 2 g[n - 2k]
* Slice s at rate f0/D_s, starting J_s full-rate taps before coalescence:
      o_s[l, k] = sum_{m < N_s} U_s[l, m] x_s[k - J_s/D_s - m]
      y_s = M_s o_s
* Up-sample-and-add from the lowest rate up: w_K = y at level K, and
  w_k = (slices at level k) + interpolate(w_{k+1}); Y = w_0.
* z_i = Y_{2i} + i Y_{2i+1}; trigger windows are [floor(w f0 a/b),
  floor((w+1) f0 a/b)) aligned to sample 0; the peak of a window is the
  lowest index attaining the maximum of |z_i|; a trigger is a window peak
  with |z| >= threshold (inclusive).

The direct form (the matched filter the method approximates) is
rho_r[n] = sum_j h_r[j] x[n - j], z = rho_{2i} + i rho_{2i+1}.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view
from scipy.signal import fftconvolve

HALF_Q = 32
KAISER_BETA = 10.0


@dataclass
class Seq:
    """values[..., i] is the sequence at absolute index start + i; zero elsewhere."""

    values: np.ndarray
    start: int

    @property
    def stop(self) -> int:
        return self.start + self.values.shape[-1]

    def window(self, lo: int, hi: int) -> np.ndarray:
        """Values on [lo, hi) with zeros outside the stored support."""
        out = np.zeros(self.values.shape[:-1] + (hi - lo,))
        a = max(lo, self.start)
        b = min(hi, self.stop)
        if b > a:
            out[..., a - lo:b - lo] = self.values[..., a - self.start:b - self.start]
        return out


def halfband_taps(q: int = HALF_Q, beta: float = KAISER_BETA) -> np.ndarray:
    """g[n] for n = -q..q (array index n + q): Kaiser-windowed half-band sinc."""
    n = np.arange(-q, q + 1, dtype=np.float64)
    win = np.i0(beta * np.sqrt(1.0 - (n / q) ** 2)) / np.i0(beta)
    # sinc(n/2) vanishes exactly at even n != 0; sin(k pi) in floating point does not
    sinc = np.where((n % 2 == 0) & (n != 0), 0.0, np.sinc(n / 2.0))
    return 0.5 * sinc * win


def _conv(u: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Full linear convolution along the last axis."""
    if u.ndim == 1:
        return np.convolve(u, k)
    return fftconvolve(u, k[None, :], mode="full", axes=-1)


def decimate2(u: Seq, g: np.ndarray | None = None) -> Seq:
    """d[k] = sum_{|n|<=Q} g[n] u[2k - n] on its whole (finite) support."""
    g = halfband_taps() if g is None else g
    q = (g.shape[0] - 1) // 2
    full = _conv(u.values, g)            # full[i] is the sum at 2k = u.start - q + i
    p0 = u.start - q
    i0 = 0 if p0 % 2 == 0 else 1
    return Seq(np.ascontiguousarray(full[..., i0::2]), (p0 + i0) // 2)


def interpolate2(w: Seq, g: np.ndarray | None = None) -> Seq:
    """v[n] = sum_k w[k] 2 g[n - 2k] on its whole support."""
    g = halfband_taps() if g is None else g
    q = (g.shape[0] - 1) // 2
    n = w.values.shape[-1]
    z = np.zeros(w.values.shape[:-1] + (2 * n - 1,))
    z[..., 0::2] = w.values               # zero-stuffed: z at 2*(w.start + k)
    return Seq(_conv(z, 2.0 * g), 2 * w.start - q)


def fir(basis: np.ndarray, x: Seq, shift: int, k_lo: int, k_hi: int, chunk: int = 8192) -> np.ndarray:
    """o[l, k] = sum_{m < N} basis[l, m] x[k - shift - m] for k in [k_lo, k_hi)."""
    n_taps = basis.shape[1]
    out = np.empty((basis.shape[0], k_hi - k_lo))
    rev = np.ascontiguousarray(basis[:, ::-1])       # rev[l, m'] = basis[l, N-1-m']
    # the windows are copied out contiguously so that the dot products run in
    # BLAS; a copy holds at most 2^27 values (long filters take fewer outputs)
    chunk = max(1, min(chunk, (1 << 27) // n_taps))
    for c0 in range(k_lo, k_hi, chunk):
        c1 = min(k_hi, c0 + chunk)
        xs = x.window(c0 - shift - n_taps + 1, c1 - shift)
        # win[k', m'] = x[c0 - shift - N + 1 + k' + m']
        win = np.ascontiguousarray(sliding_window_view(xs, n_taps))
        out[:, c0 - k_lo:c1 - k_lo] = rev @ win.T
    return out


def _level(bank, s: int) -> int:
    d = bank.f0 // bank.slices[s].rate
    return int(d).bit_length() - 1


def level_ranges(n_lo: int, n_hi: int, n_levels: int, q: int = HALF_Q):
    """Index range needed at every level for full-rate outputs [n_lo, n_hi).

    Interpolation reads w[k] for |n - 2k| <= q, so level k+1 must cover
    [ceil((lo - q)/2), floor((hi - 1 + q)/2) + 1).
    """
    need = [(n_lo, n_hi)]
    for _ in range(1, n_levels):
        lo, hi = need[-1]
        need.append((-((q - lo) // 2), (hi - 1 + q) // 2 + 1))
    return need


def lloid_snr(bank, x: np.ndarray, n_lo: int = 0, n_hi: int | None = None,
              templates: np.ndarray | None = None, return_real: bool = False):
    """Complex SNR z[i, n] of the SVD multi-rate form for n in [n_lo, n_hi).

    bank: an SVD bank (f0, slices with rate/start_tap/basis/mixing).
    x: full-rate strain on [0, T).  templates: optional subset of template ids.
    """
    if n_hi is None:
        n_hi = x.shape[0]
    g = halfband_taps()
    if templates is None:
        templates = np.arange(bank.n_templates)
    rows = np.empty(2 * len(templates), dtype=np.int64)
    rows[0::2] = 2 * np.asarray(templates)
    rows[1::2] = 2 * np.asarray(templates) + 1

    n_levels = 1 + max(_level(bank, s) for s in range(len(bank.slices)))
    need = level_ranges(n_lo, n_hi, n_levels)

    # down-sampled strain at every level, on its whole support
    xs = [Seq(np.asarray(x, dtype=np.float64), 0)]
    for _ in range(1, n_levels):
        xs.append(decimate2(xs[-1], g))

    # slice outputs y_s = M_s o_s on the range its level needs
    y_at = [None] * n_levels
    for s, sl in enumerate(bank.slices):
        k = _level(bank, s)
        d = bank.f0 // sl.rate
        lo, hi = need[k]
        o = fir(sl.basis, xs[k], sl.start_tap // d, lo, hi)
        y = sl.mixing[rows] @ o
        y_at[k] = y if y_at[k] is None else y_at[k] + y

    # up-sample and add, lowest rate first
    w = None
    for k in range(n_levels - 1, -1, -1):
        lo, hi = need[k]
        acc = np.zeros((rows.shape[0], hi - lo))
        if w is not None:
            acc += interpolate2(w, g).window(lo, hi)
        if y_at[k] is not None:
            acc += y_at[k]
        w = Seq(acc, lo)
    y_full = w.values
    if return_real:
        return y_full
    return y_full[0::2] + 1j * y_full[1::2]


def direct_snr(filters: np.ndarray, x: np.ndarray, n_lo: int = 0, n_hi: int | None = None):
    """Exact matched filter rho_r[n] = sum_j h_r[j] x[n - j], as complex z [F, n].

    filters: [2F, N] with row 2i = cos, 2i+1 = sin filter of template i.
    """
    if n_hi is None:
        n_hi = x.shape[0]
    n_taps = filters.shape[1]
    xs = Seq(np.asarray(x, dtype=np.float64), 0).window(n_lo - n_taps + 1, n_hi)
    full = _conv(filters, xs) if filters.shape[0] > 1 else np.convolve(filters[0], xs)[None]
    # full[r, i] = sum_j h_r[j] xs[i - j] = rho at n = n_lo - N + 1 + i
    rho = full[:, n_taps - 1:n_taps - 1 + (n_hi - n_lo)]
    return rho[0::2] + 1j * rho[1::2]


def window_starts(n_windows: int, f0: int, num: int, den: int) -> np.ndarray:
    """First sample of windows 0..n_windows (inclusive end marker)."""
    w = np.arange(n_windows + 1, dtype=np.int64)
    return (w * f0 * num) // den


def window_index(n: np.ndarray, f0: int, num: int, den: int) -> np.ndarray:
    """Window containing each sample n >= 0."""
    n = np.asarray(n, dtype=np.int64)
    top = int(n.max()) if n.size else 0
    n_w = (top + 1) * den // (f0 * num) + 2
    starts = window_starts(n_w, f0, num, den)
    return np.searchsorted(starts, n, side="right") - 1


def peak_table(z: np.ndarray, n_lo: int, f0: int, num: int, den: int):
    """Per (template, window) maximum of |z| over the samples present.

    z: complex [F, n] for samples n_lo .. n_lo + n - 1.  Windows that
    intersect this range are reported, each over its intersection.
    Returns (windows [W], peak_abs [F, W], peak_sample [F, W], peak_phase [F, W]).
    """
    n_hi = n_lo + z.shape[1]
    w_first = int(window_index(np.array([n_lo]), f0, num, den)[0])
    w_last = int(window_index(np.array([n_hi - 1]), f0, num, den)[0])
    starts = window_starts(w_last + 1, f0, num, den)
    wins = np.arange(w_first, w_last + 1)
    absz = np.abs(z)
    pa = np.empty((z.shape[0], wins.shape[0]))
    ps = np.empty((z.shape[0], wins.shape[0]), dtype=np.int64)
    ph = np.empty((z.shape[0], wins.shape[0]))
    for c, w in enumerate(wins):
        a = max(int(starts[w]), n_lo) - n_lo
        b = min(int(starts[w + 1]), n_hi) - n_lo
        seg = absz[:, a:b]
        arg = np.argmax(seg, axis=1)                  # first occurrence = lowest index
        pa[:, c] = seg[np.arange(z.shape[0]), arg]
        ps[:, c] = n_lo + a + arg
        zz = z[np.arange(z.shape[0]), a + arg]
        ph[:, c] = np.arctan2(zz.imag, zz.real)
    return wins, pa, ps, ph


def triggers(z: np.ndarray, n_lo: int, f0: int, num: int, den: int, threshold: float = 4.0,
             templates: np.ndarray | None = None):
    """Window peaks with |z| >= threshold: list of (template, window, sample, snr, phase)."""
    wins, pa, ps, ph = peak_table(z, n_lo, f0, num, den)
    ids = np.arange(z.shape[0]) if templates is None else np.asarray(templates)
    out = []
    for r in range(z.shape[0]):
        for c in range(wins.shape[0]):
            if pa[r, c] >= threshold:
                out.append((int(ids[r]), int(wins[c]), int(ps[r, c]), float(pa[r, c]), float(ph[r, c])))
    return out


def subsample_peak(a_prev, a_peak, a_next):
    """Sub-sample refinement of a sampled maximum (Sec. III.C names sub-sample
    interpolation at the SNR peak as the feature behind the port's slightly
    lower network SNRs).  The parabola through (-1, a_prev), (0, a_peak),
    (+1, a_next) has its vertex at

        dt = (a_prev - a_next) / (2 (a_prev - 2 a_peak + a_next)),

    with value a_peak - (a_prev - a_next) dt / 4.  dt is clipped to
    [-1/2, 1/2]; a flat or convex triple (curvature >= 0) keeps dt = 0 and
    the sampled value.  Applied to |z|.  Arrays broadcast; returns (dt, value)."""
    a_prev, a_peak, a_next = (np.asarray(v, dtype=np.float64) for v in (a_prev, a_peak, a_next))
    curv = a_prev - 2.0 * a_peak + a_next
    ok = curv < 0.0
    dt = np.where(ok, (a_prev - a_next) / np.where(ok, 2.0 * curv, 1.0), 0.0)
    dt = np.clip(dt, -0.5, 0.5)
    value = np.where(ok, a_peak - 0.25 * (a_prev - a_next) * dt, a_peak)
    return dt, value


def xi2(z: np.ndarray, n_lo: int, n_end: int, n_star: int, acorr: np.ndarray) -> float:
    """Signal-consistency value of one peak (Sec. II.A computes it, with the
    phase, for every trigger, citing the autocorrelation test of the GstLAL
    papers).  Restated: with the template's normalised complex
    autocorrelation R[k], k = -K..K (R[0] = 1), a signal matching the template
    makes the SNR around the peak follow z[n* + k] = z[n*] R[k], so

        xi2 = sum_k |z[n* + k] - z[n*] R[k]|^2 / sum_k (2 - 2 |R[k]|^2),

    the denominator being the expected numerator in unit white noise (E|z|^2
    = 2 for unit-norm cos and sin filters), so that xi2 averages 1 on noise.
    Both sums run over the lags with 0 <= n* + k < n_end (the samples the SNR
    series has); a zero denominator gives 0.

    z: complex SNR of the template on samples n_lo .. n_lo + len - 1, covering
    the lags used; acorr: complex [2K + 1], index K + k for lag k."""
    half = (acorr.shape[0] - 1) // 2
    lag = np.arange(-half, half + 1)
    n = n_star + lag
    ok = (n >= 0) & (n < n_end)
    zk = z[n[ok] - n_lo]
    r = acorr[ok]
    zs = z[n_star - n_lo]
    num = float(np.sum(np.abs(zk - zs * r) ** 2))
    den = float(np.sum(2.0 - 2.0 * np.abs(r) ** 2))
    return num / den if den > 0.0 else 0.0


def sigma2(bank) -> np.ndarray:
    """Squared full-rate norm of each reconstructed template (cos + sin).

    Slice s reconstructs rows 2i, 2i+1 as M_s U_s at rate f0/D_s with
    orthonormal basis rows, so their squared norm is sum_l M_s[r, l]^2; each
    low-rate sample carries weight D_s, so the full-rate norm is that sum
    divided by D_s.  sigma2_i = sum_s (1/D_s) sum_l (M_s[2i,l]^2 + M_s[2i+1,l]^2).
    """
    out = np.zeros(bank.n_templates)
    for sl in bank.slices:
        d = bank.f0 // sl.rate
        m2 = (sl.mixing ** 2).sum(axis=1)
        out += (m2[0::2] + m2[1::2]) / d
    return out
