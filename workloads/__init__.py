"""Seeded synthetic inputs for the LLOID filtering path.

This package generates the *inputs* of the filtering path and nothing else:
closed-form chirp templates, the time-sliced SVD bank built from them (the
setup stage that precedes filtering, Sec. II.A of the paper) with the
templates' autocorrelations (the input of the signal-consistency value), white Gaussian
strain and injected signals.  It holds none of the filtering arithmetic
(resampling, correlation, mixing, up-sample/add, peak finding); the FP64
oracle and the HIP library each implement that on their own.
"""

from .chirp import ChirpFamily, mass_chirps, duration_chirps
from .bank import SvdBank, BankSlice, SliceSpec, build_svd_bank, slice_matrix, autocorrelation, bank_autocorrelation
from .strain import white_noise, Injection, inject, draw_injections, add_waveform
from . import configs

__all__ = [
    "ChirpFamily", "mass_chirps", "duration_chirps",
    "SvdBank", "BankSlice", "SliceSpec", "build_svd_bank", "slice_matrix", "autocorrelation",
    "bank_autocorrelation",
    "white_noise", "Injection", "inject", "draw_injections", "add_waveform", "configs",
]
