"""White Gaussian strain and injected chirp signals.

The paper's computational benchmark filters white Gaussian data (Sec. IV);
whitened strain of unit variance per full-rate sample stands in for the
conditioned detector data.  An injection of template i with coalescence at
integer sample t0, phase phi and target amplitude A adds

    s[t0 - j] = A * g[j] / ||g||,   g = cos(phi) h_cos_i + sin(phi) h_sin_i

for every full-rate tap j of the template (samples before 0 are dropped).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .chirp import ChirpFamily


def white_noise(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal(n)


@dataclass
class Injection:
    template: int
    t0: int          # coalescence sample (full rate)
    snr: float       # target amplitude of the normalised waveform
    phase: float


def injection_waveform(family: ChirpFamily, inj: Injection) -> np.ndarray:
    """[n_taps] waveform indexed by tap j (samples before coalescence)."""
    n = int(family.n_full_taps()[inj.template])
    h = family.full_rate_filters(np.array([inj.template]), n_taps=n)
    g = np.cos(inj.phase) * h[0] + np.sin(inj.phase) * h[1]
    return inj.snr * g / np.linalg.norm(g)


def add_waveform(x: np.ndarray, w: np.ndarray, t0: int) -> np.ndarray:
    """x[t0 - j] += w[j] for every tap j (samples outside x are dropped); a copy."""
    x = np.array(x, dtype=np.float64, copy=True)
    j = np.arange(w.shape[0])
    n = t0 - j
    ok = (n >= 0) & (n < x.shape[0])
    x[n[ok]] += w[ok]
    return x


def inject(x: np.ndarray, family: ChirpFamily, injections) -> np.ndarray:
    x = np.array(x, dtype=np.float64, copy=True)
    for inj in injections:
        x = add_waveform(x, injection_waveform(family, inj), inj.t0)
    return x


def draw_injections(count: int, family: ChirpFamily, n_samples: int, f0: int,
                    first_s: float, gap_s: float, snr_lo: float, snr_hi: float,
                    rng: np.random.Generator, tail_s: float = 1.0):
    """Injections at integer samples >= first_s, at least gap_s apart."""
    lo = int(first_s * f0)
    hi = n_samples - int(tail_s * f0)
    span = hi - lo - int((count - 1) * gap_s * f0)
    if span <= 0:
        raise ValueError("not enough data for the requested injections")
    base = np.sort(rng.integers(0, span, size=count))
    t0 = lo + base + np.arange(count) * int(gap_s * f0)
    tmpl = rng.integers(0, family.n_templates, size=count)
    snr = rng.uniform(snr_lo, snr_hi, size=count)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=count)
    return [Injection(int(a), int(b), float(c), float(d)) for a, b, c, d in zip(tmpl, t0, snr, phase)]
