"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the FP64 oracle on the same seeded inputs.

Tolerances on the complex SNR (absolute), derived from the arithmetic:
* FP32 operands: only FP32 rounding in the sums.  The longest dot product of
  the path has N ~ 4000 terms (the C1 bank's lowest slice; the batched banks'
  long FIRs reach 1.3e5 but at |z| ~ 5), whose rounding error is of order
  sqrt(N) 2^-24 relative, i.e. 3.8e-6 of |z| <= 30: EPS_ABS 1e-4; the
  relative error at |z| >= 6 over the three chained sums (FIR,
  interpolation, mixing) about 3 sqrt(N) 2^-24 ~ 1e-5: REL_AT6 2e-5.
  (Measured on the 1024-template bank: 2.8e-5 absolute, 2.3e-6 relative.)
* FP16 operands: the rounded operands (x, U, o, the interpolation filter,
  M) each contribute 2^-11 relative to |z| <= ~30: EPS_ABS 3e-2.
* BF16 operands: the same with 2^-8: EPS_ABS 0.2.
The relative |z| error at oracle |z| >= 6 must stay within 1e-2 for FP16
and BF16 (the stated precision target).

A window's peak sample must equal the oracle's exactly unless the window is
a near tie: the oracle's |z| at the GPU's sample is within 2 eps of the
oracle's maximum, where eps bounds | |z_gpu| - |z_oracle| | over the window's
samples (if the GPU's maximum is at n_g and the oracle's at n_o, then
|z_o(n_o)| - |z_o(n_g)| <= 2 max_n | |z_g(n)| - |z_o(n)| |).  eps is the
measured maximum error of the precision: the complex-SNR error measured in
the same test where the test has the series, else the stated error of the
1024-template bank (EPS_TIE: its measured maxima 2.8e-5, 1.25e-2 and
7.3e-2, rounded up), whichever is larger.
"""

from __future__ import annotations

import sys

import numpy as np

EPS_ABS = {"f32": 1e-4, "f16": 3e-2, "bf16": 0.2}
REL_AT6 = {"f32": 2e-5, "f16": 1e-2, "bf16": 1e-2}
EPS_TIE = {"f32": 5e-5, "f16": 1.5e-2, "bf16": 8e-2}

_ctx = None


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def ctx():
    global _ctx
    if _ctx is None:
        import torch
        from paper_2410_16416_amd import lloid
        torch.cuda.init()
        _ctx = lloid.lloid_ctx_create(0)
    return _ctx


def run_filter(bank_obj, strain, compute, window, snr=False, threshold=4.0, bank_handle=None):
    from paper_2410_16416_amd import lloid
    b = bank_handle if bank_handle is not None else lloid.bank_from_svd(ctx(), bank_obj, compute)
    try:
        snr_out = np.zeros((bank_obj.n_templates, strain.shape[0], 2), dtype=np.float32) if snr else None
        res = lloid.lloid_filter(b, 0, strain, window=window, threshold=threshold, snr_out=snr_out, peaks=True)
    finally:
        if bank_handle is None:
            lloid.lloid_bank_destroy(b)
    return res


def compare_peaks(res, z_oracle_abs, pa, ps, compute, n_lo=0, windows=None, label="", eps_series=None):
    """Peak values within EPS_ABS; samples exact unless a near tie (2 eps, eps
    the larger of EPS_TIE and eps_series, the complex-SNR error measured in
    the same test).

    z_oracle_abs: [F, n] oracle |z| on samples n_lo..; pa/ps: oracle peak table
    for the windows `windows` (indices into the GPU table)."""
    eps = EPS_ABS[compute]
    tie = max(EPS_TIE[compute], eps_series or 0.0)
    g_snr = res.peak_snr if windows is None else res.peak_snr[:, windows]
    g_n = res.peak_sample if windows is None else res.peak_sample[:, windows]
    d = np.abs(g_snr - pa)
    assert np.all(np.isfinite(g_snr)), label
    assert d.max() <= eps, f"{label}: peak |z| differs by {d.max():.3e} > {eps}"
    mism = g_n != ps
    n_tie = 0
    if mism.any():
        r, c = np.nonzero(mism)
        at_gpu = z_oracle_abs[r, g_n[r, c] - n_lo]
        gap = pa[r, c] - at_gpu
        assert np.all(gap <= 2 * tie), (
            f"{label}: {int((gap > 2 * tie).sum())} peak samples differ outside near ties "
            f"(max gap {gap.max():.3e}, tie bound {2 * tie:.3e})")
        n_tie = int(mism.sum())
    return {"max_abs_peak": float(d.max()), "near_ties": n_tie, "windows": int(pa.size)}


def compare_series(z_gpu, z_oracle, compute, label=""):
    eps = EPS_ABS[compute]
    d = np.abs(z_gpu - z_oracle)
    assert np.all(np.isfinite(z_gpu)), label
    assert d.max() <= eps, f"{label}: complex SNR differs by {d.max():.3e} > {eps}"
    a = np.abs(z_oracle)
    m = a >= 6.0
    rel = 0.0
    if m.any():
        rel = float((np.abs(np.abs(z_gpu[m]) - a[m]) / a[m]).max())
        assert rel <= REL_AT6[compute], f"{label}: relative |z| error {rel:.3e} at |z| >= 6"
    return {"max_abs": float(d.max()), "max_rel_at6": rel}


def record_precision(case: str, compute: str, **stats):
    """Merge measured errors into the JSON file named by LLOID_PRECISION_OUT
    (if set): {compute: {case: stats}}.  The benchmark prints these next to
    its throughput as the stated SNR error of each precision."""
    import json
    import os
    path = os.environ.get("LLOID_PRECISION_OUT")
    if not path:
        return
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault(compute, {})[case] = stats
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def gpu_complex(res):
    s = res.snr
    return s[..., 0].astype(np.float64) + 1j * s[..., 1].astype(np.float64)
