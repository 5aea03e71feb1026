"""Data conditioning before the filter (test infrastructure only).

Sec. II.A conditions the strain before filtering: it estimates the power
spectral density (PSD), whitens the strain with a running average of the
PSD, and gates away large deviations of the whitened data.  The paper gives
no further detail; the readings fixed here:

* Segments of L samples (L a power of two), hop L/2, periodic Hann window
  w[n] = sin^2(pi n / L), for which w[n] + w[n + L/2] = 1.
* PSD of a block: the mean over its segments that lie wholly inside the
  block (segment m starts at m L/2) of the one-sided periodogram
      P[f] = c_f |sum_n w[n] x[mL/2 + n] e^{-2 pi i f n / L}|^2 / (f0 sum_n w[n]^2),
  c_f = 2 except c_0 = c_{L/2} = 1 (Welch's average; the density scaling,
  so that unit-variance white noise has S[f] = 2 / f0).
* Whitening: every segment m (from m = -1, data zero outside [0, T)) is
  windowed, transformed, multiplied by the gain G[f] = 1 / sqrt(S[f] f0 / 2)
  (0 where S[f] <= 0; the bin L - f uses G[f]), transformed back, and the
  segments are overlap-added; the window sums to 1 over the overlaps, so a
  flat PSD S = 2 sigma^2 / f0 returns x / sigma exactly.
* Gating: every sample n of the whitened data with |x_w[n]| > threshold
  zeroes x_w on [n - G, n + G] (inside the data).
"""

from __future__ import annotations

import numpy as np


def hann(L: int) -> np.ndarray:
    n = np.arange(L)
    return np.sin(np.pi * n / L) ** 2


def welch_psd(x: np.ndarray, f0: int, L: int) -> np.ndarray:
    """One-sided PSD [L/2 + 1]: mean periodogram of the whole segments."""
    T = x.shape[0]
    if T < L:
        raise ValueError("the block is shorter than one segment")
    w = hann(L)
    m_count = (T - L) // (L // 2) + 1
    acc = np.zeros(L // 2 + 1)
    for m in range(m_count):
        seg = x[m * (L // 2): m * (L // 2) + L] * w
        acc += np.abs(np.fft.rfft(seg)) ** 2
    c = np.full(L // 2 + 1, 2.0)
    c[0] = c[-1] = 1.0
    return c * acc / m_count / (f0 * np.sum(w ** 2))


def whitening_gain(psd: np.ndarray, f0: int) -> np.ndarray:
    g = np.zeros_like(psd, dtype=np.float64)
    ok = psd > 0
    g[ok] = 1.0 / np.sqrt(psd[ok] * f0 / 2.0)
    return g


def whiten(x: np.ndarray, f0: int, L: int, psd: np.ndarray) -> np.ndarray:
    T = x.shape[0]
    h = L // 2
    w = hann(L)
    g = whitening_gain(psd, f0)
    out = np.zeros(T)
    for m in range(-1, (2 * (T - 1)) // L + 1):
        lo = m * h
        seg = np.zeros(L)
        a, b = max(lo, 0), min(lo + L, T)
        seg[a - lo:b - lo] = x[a:b]
        y = np.fft.irfft(np.fft.rfft(seg * w) * g, L)
        out[a:b] += y[a - lo:b - lo]
    return out


def gate(xw: np.ndarray, threshold: float, half_width: int):
    """Returns (gated copy, number of samples zeroed)."""
    out = xw.copy()
    if threshold <= 0:
        return out, 0
    mask = np.zeros(xw.shape[0], dtype=bool)
    for n in np.nonzero(np.abs(xw) > threshold)[0]:
        mask[max(n - half_width, 0):n + half_width + 1] = True
    out[mask] = 0.0
    return out, int(mask.sum())


def condition(x: np.ndarray, f0: int, L: int, gate_threshold: float = 0.0, gate_half_width: int = 0,
              psd: np.ndarray | None = None):
    """PSD (estimated from x unless given), whitened and gated strain, samples gated."""
    s = welch_psd(x, f0, L) if psd is None else np.asarray(psd, dtype=np.float64)
    xw = whiten(x, f0, L, s)
    xg, n_gated = gate(xw, gate_threshold, gate_half_width)
    return s, xg, n_gated
