"""Time-sliced SVD banks (the setup stage of Sec. II.A).

The paper splits each group of templates into time slices, each with its
own sample rate, and decomposes every slice with an SVD; the orthogonal
basis filters and the SVD coefficients (mixing matrix) of every slice form
the "SVD bank" that the filtering stage consumes.  The filtering path takes
these arrays as its input; this module only produces them.

Slice s runs at rate r_s = f0 / D_s (D_s a power of two) and covers the
full-rate taps j = J_s + m * D_s, m = 0..N_s-1 (J_s a multiple of D_s).  Its
2F x N_s template matrix is

    H_s[r, m] = D_s * h_r(tau = (J_s + m * D_s + 1) / f0)

(the factor D_s lets a dot product at rate r_s stand for the full-rate one,
since one low-rate sample stands for D_s full-rate samples).  The thin SVD
H_s = A diag(sigma) B^T is truncated to the top L_s components:
basis U_s = B^T[:L_s] (L_s x N_s), mixing M_s = A[:, :L_s] diag(sigma[:L_s])
(2F x L_s), so H_s ~= M_s U_s.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .chirp import ChirpFamily


@dataclass
class SliceSpec:
    rate: int          # r_s (Hz)
    start_tap: int     # J_s, full-rate samples before coalescence
    n_taps: int        # N_s at rate r_s
    n_basis: int       # L_s


@dataclass
class BankSlice:
    rate: int
    start_tap: int
    n_taps: int
    basis: np.ndarray            # [L, N] float64, orthonormal rows
    mixing: np.ndarray           # [2F, L] float64
    singular_values: np.ndarray  # every singular value of H_s, descending

    @property
    def n_basis(self) -> int:
        return int(self.basis.shape[0])


@dataclass
class SvdBank:
    f0: int
    n_templates: int
    slices: list = field(default_factory=list)
    family: ChirpFamily | None = None
    # normalised complex autocorrelation of each template, [F, 2K + 1] (column
    # K + k holds lag k), or None; the input of the signal-consistency value
    autocorr: np.ndarray | None = None

    def decimation(self, s: int) -> int:
        return self.f0 // self.slices[s].rate

    def describe(self) -> str:
        parts = [f"{sl.rate}Hz J={sl.start_tap} N={sl.n_taps} L={sl.n_basis}" for sl in self.slices]
        return f"F={self.n_templates} f0={self.f0} slices=[" + "; ".join(parts) + "]"

    def flops_per_det_second(self) -> float:
        """Algorithmic flops of the method per detector-second.

        FIR: 2 L_s N_s r_s; mixing at the slice rate: 2 (2F) L_s r_s.
        """
        tot = 0.0
        for sl in self.slices:
            tot += 2.0 * sl.n_basis * sl.n_taps * sl.rate
            tot += 2.0 * (2 * self.n_templates) * sl.n_basis * sl.rate
        return tot


def slice_matrix(family: ChirpFamily, f0: int, spec: SliceSpec) -> np.ndarray:
    """H_s[r, m] = D_s * h_r((J_s + m D_s + 1) / f0), [2F, N_s]."""
    d = f0 // spec.rate
    m = np.arange(spec.n_taps)
    tau = (spec.start_tap + m * d + 1.0) / f0
    return d * family.filters_at(tau)


def _svd_sign_fix(a: np.ndarray, bt: np.ndarray):
    """Make each component's largest-magnitude basis entry positive."""
    idx = np.argmax(np.abs(bt), axis=1)
    sgn = np.sign(bt[np.arange(bt.shape[0]), idx])
    sgn[sgn == 0] = 1.0
    return a * sgn[None, :], bt * sgn[:, None]


def build_svd_bank(family: ChirpFamily, f0: int, specs: list) -> SvdBank:
    bank = SvdBank(f0=f0, n_templates=family.n_templates, family=family)
    for spec in specs:
        d = f0 // spec.rate
        if f0 % spec.rate or d & (d - 1):
            raise ValueError("slice rate must be f0 / 2**k")
        if spec.start_tap % d:
            raise ValueError("start tap must be a multiple of f0 / rate")
        h = slice_matrix(family, f0, spec)
        a, sv, bt = np.linalg.svd(h, full_matrices=False)
        a, bt = _svd_sign_fix(a, bt)
        l = min(spec.n_basis, sv.shape[0])
        bank.slices.append(BankSlice(
            rate=spec.rate, start_tap=spec.start_tap, n_taps=spec.n_taps,
            basis=np.ascontiguousarray(bt[:l]),
            mixing=np.ascontiguousarray(a[:, :l] * sv[None, :l]),
            singular_values=sv.copy()))
    return bank


def autocorrelation(filters: np.ndarray, half: int) -> np.ndarray:
    """Normalised complex autocorrelation of the templates in `filters`.

    Rows 2i and 2i+1 are the cos and sin filters of template i at taps
    j = 0..N-1 before coalescence; h_i = h_2i + i h_2i+1.  For lags
    k = -half..half,

        R_i[k] = sum_j h_i[j] conj(h_i[j - k]) / sum_j |h_i[j]|^2,

    so R_i[0] = 1 and R_i[-k] = conj(R_i[k]).  This is the covariance
    E[z_i[n + k] conj(z_i[n])] / E|z_i[n]|^2 of the complex SNR in white
    noise.  Returns complex128 [F, 2 half + 1], column half + k for lag k.
    """
    h = filters[0::2] + 1j * filters[1::2]
    n = h.shape[1]
    size = 1 << int(np.ceil(np.log2(n + half + 1)))
    spec = np.fft.fft(h, size, axis=1)
    circ = np.fft.ifft(spec * np.conj(spec), axis=1)     # circ[k] = sum_j h[j] conj(h[j - k])
    lags = np.arange(-half, half + 1) % size
    r = circ[:, lags]
    return r / np.sum(np.abs(h) ** 2, axis=1)[:, None]


def bank_autocorrelation(bank: SvdBank, half: int, batch: int = 64) -> np.ndarray:
    """Autocorrelation input of a bank: from the full-rate chirp templates when
    the bank was built from a family, else (banks with random bases) from the
    reconstruction M U of its full-rate slice, which stands in for templates."""
    if bank.family is not None:
        out = np.empty((bank.n_templates, 2 * half + 1), dtype=np.complex128)
        for a in range(0, bank.n_templates, batch):
            rows = np.arange(a, min(a + batch, bank.n_templates))
            out[rows] = autocorrelation(bank.family.full_rate_filters(rows), half)
        return out
    top = bank.slices[0]
    if top.rate != bank.f0:
        raise ValueError("a bank without a family needs a full-rate first slice")
    out = np.empty((bank.n_templates, 2 * half + 1), dtype=np.complex128)
    for a in range(0, bank.n_templates, batch):
        b = min(a + batch, bank.n_templates)
        out[a:b] = autocorrelation(top.mixing[2 * a:2 * b] @ top.basis, half)
    return out
