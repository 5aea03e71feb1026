"""FP64 CPU oracle for the LLOID filtering path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The HIP library never calls it, and the
two share no code: the oracle computes every step (half-band taps,
decimation, correlation, mixing, interpolation, complex SNR, windowed
peaks, triggers, sub-sample peaks, the signal-consistency value, the
coincidence of two detectors' triggers, and the conditioning before the
filter: PSD, whitening, gating) from the paper's description in plain
NumPy/SciPy.

Parity status: every function is pinned by the CPU tests (brute force on
tiny inputs, closed forms, library routines, bounds); the absolute
accuracy of the multi-rate form against the paper's own GstLAL resampler and
slicing (not described in the paper) is parity unpinned.
"""

from .lloid import (
    Seq, halfband_taps, decimate2, interpolate2, fir, lloid_snr, direct_snr,
    window_index, window_starts, peak_table, triggers, sigma2, level_ranges, subsample_peak, xi2,
)

from .coinc import coincidences
from .condition import welch_psd, whiten, gate, condition, hann

__all__ = [
    "Seq", "halfband_taps", "decimate2", "interpolate2", "fir", "lloid_snr",
    "direct_snr", "window_index", "window_starts", "peak_table", "triggers",
    "sigma2", "level_ranges", "subsample_peak", "xi2", "coincidences",
    "welch_psd", "whiten", "gate", "condition", "hann",
]
