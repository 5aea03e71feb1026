"""Seeded workload recipes.

Each recipe returns a bank and per-detector strain with the shapes of the
paper's workloads (white Gaussian data, ~1000-template banks, Sec. IV) and
of the configurations the implementation is measured on:

  plain_c0   single rate 1024 Hz, 64 mass chirps (1 s, 1024 taps), SVD to 32
             basis filters; 8 s of noise, one injection at SNR 10 at sample
             4146 with phase 0; 0.1 s trigger windows.
  multirate_c1
             f0 = 2048, 1024 duration chirps (0.5-32 s, f_low = 4), slices
             2048/512/128 Hz over tau in [0,0.5)/[0.5,4)/[4,32) s with
             200/150/100 basis filters; 2 detectors of noise with 20
             injections, SNR U[6,30]; 1 s windows.
  mini_multirate
             a small three-slice bank (16 templates, f0 = 1024, rates
             1024/256/64) for fast parity tests; it skips levels 512 and 128.
  batched_banks
             uneven banks: F ~ U{200..2000}, 1-4 slices at 2048 plus distinct
             rates from {1024, 512, 256, 128}, lengths 0.5-64 s.

Seeds: noise of detector d in recipe c uses SEED0 + 10 c + d; the bank
uses SEED0 + 10 c + 9 and the injections SEED0 + 10 c + 8.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .bank import SliceSpec, SvdBank, build_svd_bank
from .chirp import duration_chirps, mass_chirps
from .strain import Injection, draw_injections, inject, white_noise

SEED0 = 2410164160


def seed(config: int, slot: int) -> int:
    return SEED0 + 10 * config + slot


@dataclass
class Workload:
    name: str
    bank: SvdBank
    strains: list            # per detector, float64 arrays (noise + injections)
    injections: list
    window_num: int
    window_den: int
    threshold: float = 4.0
    extra: dict = field(default_factory=dict)

    @property
    def n_samples(self) -> int:
        return int(self.strains[0].shape[0])


# ---------------------------------------------------------------- plain (C0)

def plain_c0_bank() -> SvdBank:
    rng = np.random.default_rng(seed(0, 9))
    fam = mass_chirps(64, 1024, 1.0, 20.0, 1.0, 3.0, rng)
    return build_svd_bank(fam, 1024, [SliceSpec(1024, 0, 1024, 32)])


def plain_c0(seconds: int = 8, detectors: int = 1, bank: SvdBank | None = None) -> Workload:
    bank = bank or plain_c0_bank()
    n = seconds * bank.f0
    tmpl = int(np.random.default_rng(seed(0, 8)).integers(0, bank.n_templates))
    injs = [Injection(template=tmpl, t0=4146, snr=10.0, phase=0.0)] if n > 4146 else []
    strains = []
    for d in range(detectors):
        x = white_noise(n, np.random.default_rng(seed(0, d)))
        strains.append(inject(x, bank.family, injs))
    return Workload("plain_c0", bank, strains, injs, 1, 10)


# ------------------------------------------------------------ multirate (C1)

C1_SLICES = [SliceSpec(2048, 0, 1024, 200), SliceSpec(512, 1024, 1792, 150),
             SliceSpec(128, 8192, 3584, 100)]


def multirate_c1_bank(n_templates: int = 1024) -> SvdBank:
    rng = np.random.default_rng(seed(1, 9))
    fam = duration_chirps(n_templates, 2048, 0.5, 32.0, 4.0, rng)
    return build_svd_bank(fam, 2048, C1_SLICES)


def multirate_c1(seconds: int = 1024, detectors: int = 2, n_injections: int = 20,
                 bank: SvdBank | None = None) -> Workload:
    bank = bank or multirate_c1_bank()
    n = seconds * bank.f0
    injs = []
    if n_injections:
        injs = draw_injections(n_injections, bank.family, n, bank.f0, first_s=32.0, gap_s=2.0,
                               snr_lo=6.0, snr_hi=30.0, rng=np.random.default_rng(seed(1, 8)))
    strains = [inject(white_noise(n, np.random.default_rng(seed(1, d))), bank.family, injs)
               for d in range(detectors)]
    return Workload("multirate_c1", bank, strains, injs, 1, 1)


# ------------------------------------------------------------ small multirate

MINI_SLICES = [SliceSpec(1024, 0, 256, 24), SliceSpec(256, 256, 192, 16),
               SliceSpec(64, 1024, 192, 12)]


def mini_multirate_bank() -> SvdBank:
    rng = np.random.default_rng(seed(5, 9))
    fam = duration_chirps(16, 1024, 0.25, 4.0, 4.0, rng)
    return build_svd_bank(fam, 1024, MINI_SLICES)


def mini_multirate(seconds: int = 12, detectors: int = 1, n_injections: int = 2,
                   bank: SvdBank | None = None) -> Workload:
    bank = bank or mini_multirate_bank()
    n = seconds * bank.f0
    injs = draw_injections(n_injections, bank.family, n, bank.f0, first_s=4.0, gap_s=1.0,
                           snr_lo=8.0, snr_hi=20.0, rng=np.random.default_rng(seed(5, 8))) \
        if n_injections else []
    strains = [inject(white_noise(n, np.random.default_rng(seed(5, d))), bank.family, injs)
               for d in range(detectors)]
    return Workload("mini_multirate", bank, strains, injs, 1, 4)


# --------------------------------------------------------- batched banks (C3)

BATCH_RATES = (1024, 512, 256, 128)


def draw_bank_specs(rng: np.random.Generator, f0: int = 2048):
    """Draw one uneven bank: (F, durations' upper end, slice specs).

    F ~ U{200..2000}; S ~ U{1..4}; rates are f0 plus S-1 distinct draws from
    {1024, 512, 256, 128}, descending.  D_max ~ logU[0.5, 64] s.  Slice
    boundaries are geometric, tau_k = D_max * 8**-(S-k), snapped to 1/128 s.
    A slice that ends up empty or shorter than 50 taps merges with its
    lower-rate neighbour (the last slice with its higher-rate one); the
    merged span keeps the higher of the two rates so that no part of a
    template is sampled below the rate it was assigned.
    L_s ~ U{50..400}, clipped to min(2F, N_s).
    """
    n_t = int(rng.integers(200, 2001))
    n_s = int(rng.integers(1, 5))
    rates = [f0] + sorted(rng.choice(BATCH_RATES, size=n_s - 1, replace=False).tolist(), reverse=True)
    d_max = float(np.exp(rng.uniform(np.log(0.5), np.log(64.0))))
    d_max = max(np.floor(d_max * 128.0) / 128.0, 1.0 / 128.0)
    bounds = [0.0] + [np.floor(d_max * 8.0 ** (-(n_s - k)) * 128.0) / 128.0 for k in range(1, n_s)] + [d_max]
    edges = list(bounds)
    rr = list(rates)
    k = 0
    while k < len(rr):
        taps = int(round((edges[k + 1] - edges[k]) * rr[k]))
        if taps < 50 and len(rr) > 1:
            if k + 1 < len(rr):
                del edges[k + 1]   # slice k absorbs slice k+1's span at rate rr[k]
                del rr[k + 1]
            else:
                del edges[k]       # the last slice joins the one above it
                del rr[k]
            continue
        k += 1
    specs = []
    for k, r in enumerate(rr):
        d = f0 // r
        j = int(round(edges[k] * f0))
        j -= j % d
        end = int(round(edges[k + 1] * f0))
        n_taps = (end - j + d - 1) // d
        lb = int(rng.integers(50, 401))
        specs.append(SliceSpec(r, j, n_taps, min(lb, 2 * n_t, n_taps)))
    return n_t, d_max, specs


def batched_bank(index: int, config: int = 3, f0: int = 2048) -> SvdBank:
    rng = np.random.default_rng(seed(config, 9) + 1000 * index)
    n_t, d_max, specs = draw_bank_specs(rng, f0)
    fam = duration_chirps(n_t, f0, d_max / 4.0, d_max, 4.0, rng)
    return build_svd_bank(fam, f0, specs)


def small_uneven_bank(index: int, f0: int = 1024) -> SvdBank:
    """A small bank with the batched recipe's structure (1-4 slices at f0 and
    distinct lower rates, uneven template count and basis sizes), short enough
    for the oracle: F ~ U{8..40}, D_max ~ logU[0.5, 3] s."""
    rng = np.random.default_rng(seed(6, 9) + 1000 * index)
    n_t = int(rng.integers(8, 41))
    rates_all = (f0 // 2, f0 // 4, f0 // 8, f0 // 16)
    n_s = int(rng.integers(1, 5))
    rates = [f0] + sorted(rng.choice(rates_all, size=n_s - 1, replace=False).tolist(), reverse=True)
    d_max = float(np.floor(np.exp(rng.uniform(np.log(0.5), np.log(3.0))) * 64) / 64)
    edges = [0.0] + [np.floor(d_max * 4.0 ** (-(n_s - k)) * 64) / 64 for k in range(1, n_s)] + [d_max]
    specs = []
    for k, r in enumerate(rates):
        d = f0 // r
        j = int(round(edges[k] * f0))
        j -= j % d
        end = int(round(edges[k + 1] * f0))
        n_taps = max((end - j + d - 1) // d, 1)
        lb = int(rng.integers(4, 24))
        specs.append(SliceSpec(r, j, n_taps, max(1, min(lb, 2 * n_t, n_taps))))
    fam = duration_chirps(n_t, f0, d_max / 2.0, d_max, 3.0, rng)
    return build_svd_bank(fam, f0, specs)


def random_basis_bank(n_templates: int, specs, f0: int, rng: np.random.Generator) -> SvdBank:
    """A bank with the given shape whose bases are seeded random orthonormal rows
    and whose mixing entries are Gaussian with the per-column energy of an SVD
    bank (decreasing singular values).  The filtering work depends only on the
    shapes, so this stands in for chirp SVD banks whose construction would take
    minutes (a 4000 x 131072 decomposition for a 64 s single-slice bank)."""
    from .bank import BankSlice
    bank = SvdBank(f0=f0, n_templates=n_templates)
    for sp in specs:
        q, _ = np.linalg.qr(rng.standard_normal((sp.n_taps, sp.n_basis)))
        sv = np.sqrt(2.0 * n_templates / sp.n_basis) * np.exp(-np.arange(sp.n_basis) / max(sp.n_basis, 1))
        mix = rng.standard_normal((2 * n_templates, sp.n_basis)) * (sv / np.sqrt(2.0 * n_templates))[None, :]
        bank.slices.append(BankSlice(rate=sp.rate, start_tap=sp.start_tap, n_taps=sp.n_taps,
                                     basis=np.ascontiguousarray(q.T), mixing=mix, singular_values=sv))
    return bank


def batched_c3_bank(index: int, f0: int = 2048) -> SvdBank:
    """Bank `index` of the batched measurement: shape drawn by draw_bank_specs,
    values from random_basis_bank."""
    rng = np.random.default_rng(seed(3, 9) + 1000 * index)
    n_t, d_max, specs = draw_bank_specs(rng, f0)
    return random_basis_bank(n_t, specs, f0, rng)


def batched_c3_banks(n_banks: int = 64, f0: int = 2048):
    """Uneven banks for the batched measurement (banks 0 .. n_banks - 1)."""
    return [batched_c3_bank(i, f0) for i in range(n_banks)]


def longest_c3_bank(f0: int = 2048) -> SvdBank:
    """The batched recipe's extreme FIR shape: one slice at f0 with the longest
    filter (64 s, 131072 taps), the most basis filters (400) and the most
    templates (2000); random orthonormal basis as in random_basis_bank."""
    rng = np.random.default_rng(seed(3, 7))
    return random_basis_bank(2000, [SliceSpec(f0, 0, 64 * f0, 400)], f0, rng)


def reconstructed_waveform(bank: SvdBank, template: int, phase: float = 0.0) -> np.ndarray:
    """Template `template` of a single-slice bank at the full rate, as its SVD
    bank reconstructs it (row r of M U; tap m is m samples before
    coalescence): cos(phase) h_cos + sin(phase) h_sin, unit-normalised.  An
    injection for banks without a chirp family (random bases)."""
    if len(bank.slices) != 1 or bank.slices[0].rate != bank.f0 or bank.slices[0].start_tap != 0:
        raise ValueError("needs a single slice at the full rate starting at tap 0")
    sl = bank.slices[0]
    h = sl.mixing[[2 * template, 2 * template + 1]] @ sl.basis
    g = np.cos(phase) * h[0] + np.sin(phase) * h[1]
    return g / np.linalg.norm(g)
