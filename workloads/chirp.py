"""Closed-form leading-order chirp templates.

The paper's banks are built from LAL waveform models that are not available
here; these stand in for them.  Every template follows the leading-order
(Newtonian) chirp law in time-to-coalescence tau > 0:

    f(tau)   = c * tau**(-3/8)
    Phi(tau) = -(16 pi / 5) * c * tau**(5/8)      (the integral of -2 pi f)
    A(tau)   = f(tau)**(2/3)

and is zero for tau > D (its duration).  Full-rate tap j (j = 0, 1, ...)
sits at tau_j = (j + 1) / f0, i.e. j counts samples before coalescence.
Each template i gives two real filters, cos (row 2i) and sin (row 2i+1),
each scaled to unit norm over its full-rate taps.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ChirpFamily:
    """A set of F chirps sharing the tau**(-3/8) law.

    coef[i]     : c_i in f = c_i * tau**(-3/8)
    duration[i] : D_i in seconds; the template is zero for tau > D_i
    f0          : full sample rate (Hz)
    """

    coef: np.ndarray
    duration: np.ndarray
    f0: int

    def __post_init__(self):
        self.coef = np.asarray(self.coef, dtype=np.float64)
        self.duration = np.asarray(self.duration, dtype=np.float64)
        self._norm = None

    @property
    def n_templates(self) -> int:
        return int(self.coef.shape[0])

    def n_full_taps(self) -> np.ndarray:
        """Full-rate taps of each template: the j with (j+1)/f0 <= D_i."""
        return np.floor(self.duration * self.f0 + 1e-9).astype(np.int64)

    def max_full_taps(self) -> int:
        return int(self.n_full_taps().max())

    def _raw(self, rows: np.ndarray, tau: np.ndarray):
        """Unnormalised cos and sin parts at time-to-coalescence tau.

        rows: template indices [R]; tau: [R, T] or [T] (seconds, > 0).
        """
        c = self.coef[rows][:, None]
        d = self.duration[rows][:, None]
        tau = np.broadcast_to(tau, (rows.shape[0],) + np.shape(tau)[-1:])
        f = c * tau ** (-3.0 / 8.0)
        amp = f ** (2.0 / 3.0)
        phase = -(16.0 * np.pi / 5.0) * c * tau ** (5.0 / 8.0)
        inside = tau <= d + 1e-12
        hc = np.where(inside, amp * np.cos(phase), 0.0)
        hs = np.where(inside, amp * np.sin(phase), 0.0)
        return hc, hs

    def norms(self) -> np.ndarray:
        """[F, 2] full-rate L2 norms of the raw cos and sin parts."""
        if self._norm is None:
            F = self.n_templates
            out = np.zeros((F, 2))
            n_tap = self.max_full_taps()
            chunk = 8192
            rows = np.arange(F)
            for j0 in range(0, n_tap, chunk):
                j = np.arange(j0, min(n_tap, j0 + chunk))
                tau = (j + 1.0) / self.f0
                hc, hs = self._raw(rows, tau)
                out[:, 0] += np.einsum("ij,ij->i", hc, hc)
                out[:, 1] += np.einsum("ij,ij->i", hs, hs)
            self._norm = np.sqrt(out)
        return self._norm

    def filters_at(self, tau: np.ndarray, rows: np.ndarray | None = None) -> np.ndarray:
        """Unit-norm real filters evaluated at tau.

        Returns [2R, T]: row 2k is the cos filter of template rows[k], row
        2k+1 its sin filter.  Normalisation is over the full-rate taps.
        """
        if rows is None:
            rows = np.arange(self.n_templates)
        rows = np.asarray(rows)
        hc, hs = self._raw(rows, np.asarray(tau, dtype=np.float64))
        nrm = self.norms()[rows]
        out = np.empty((2 * rows.shape[0], hc.shape[-1]))
        out[0::2] = hc / nrm[:, 0:1]
        out[1::2] = hs / nrm[:, 1:2]
        return out

    def full_rate_filters(self, rows: np.ndarray | None = None, n_taps: int | None = None) -> np.ndarray:
        """[2R, n_taps] unit-norm filters at full-rate taps j = 0..n_taps-1."""
        if n_taps is None:
            n_taps = self.max_full_taps()
        j = np.arange(n_taps)
        return self.filters_at((j + 1.0) / self.f0, rows)


def mass_chirps(n_templates: int, f0: int, duration_s: float, k_const: float,
                mc_lo: float, mc_hi: float, rng: np.random.Generator) -> ChirpFamily:
    """Chirps parameterised by chirp mass: f = K * Mc**(-5/8) * tau**(-3/8).

    Mc ~ U[mc_lo, mc_hi] (arbitrary units); every template spans duration_s.
    """
    mc = rng.uniform(mc_lo, mc_hi, size=n_templates)
    coef = k_const * mc ** (-5.0 / 8.0)
    dur = np.full(n_templates, float(duration_s))
    return ChirpFamily(coef=coef, duration=dur, f0=f0)


def duration_chirps(n_templates: int, f0: int, dur_lo: float, dur_hi: float,
                    f_low: float, rng: np.random.Generator) -> ChirpFamily:
    """Chirps parameterised by duration: f = f_low * (tau / D)**(-3/8), tau <= D.

    D ~ log-uniform on [dur_lo, dur_hi]; at tau = D the frequency is f_low.
    Durations are snapped down to a whole number of full-rate samples.
    """
    d = np.exp(rng.uniform(np.log(dur_lo), np.log(dur_hi), size=n_templates))
    d = np.floor(d * f0) / f0
    coef = f_low * d ** (3.0 / 8.0)
    return ChirpFamily(coef=coef, duration=d, f0=f0)
