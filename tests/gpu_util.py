"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the FP64 oracle on the same seeded inputs.

Tolerances (absolute, on |z| and on the complex SNR), derived from the
operand precision (the rounded operands each contribute their type's unit
roundoff relative to |z| <= ~30, over dot products of ~500 terms): FP32
operands 2e-3; FP16 operands 3e-2; BF16 operands 0.2.  The relative |z| error at oracle |z| >= 6 must stay within
1e-2 for FP16 and BF16 (the stated precision target) and 1e-4 for FP32.
A window's peak sample must equal the oracle's exactly unless the window is
a near tie: the oracle's |z| at the GPU's sample is within 2 eps_abs of the
oracle's maximum.
"""

from __future__ import annotations

import sys

import numpy as np

EPS_ABS = {"f32": 2e-3, "f16": 3e-2, "bf16": 0.2}
REL_AT6 = {"f32": 1e-4, "f16": 1e-2, "bf16": 1e-2}

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


def compare_peaks(res, z_oracle_abs, pa, ps, compute, n_lo=0, windows=None, label=""):
    """Peak values within eps_abs; samples exact unless a near tie.

    z_oracle_abs: [F, n] oracle |z| on samples n_lo..; pa/ps: oracle peak table
    for the windows `windows` (indices into the GPU table)."""
    eps = EPS_ABS[compute]
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
        assert np.all(gap <= 2 * eps), (
            f"{label}: {int((gap > 2 * eps).sum())} peak samples differ outside near ties "
            f"(max gap {gap.max():.3e})")
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
