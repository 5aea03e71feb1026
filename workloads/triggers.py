"""Seeded synthetic trigger lists of two detectors, for the coincidence step.

Records have the 48-byte trigger layout; each list is sorted by (bank,
template, sample) as a filter call returns it: per (bank, template, window)
a trigger with probability `rate` at a uniform sample of the window.  The
second detector repeats a share `shared` of the first detector's triggers,
moved by a uniform offset of at most `spread` samples (kept inside the same
window), and adds its own.  No filtering arithmetic happens here.
"""

from __future__ import annotations

import numpy as np

TRIGGER_FIELDS = [("bank", np.int32), ("detector", np.int32), ("template_id", np.int32),
                  ("xi2", np.float32), ("window", np.int64), ("sample", np.int64),
                  ("snr", np.float32), ("phase", np.float32), ("snr_interp", np.float32),
                  ("dt", np.float32)]
TRIGGER_DTYPE = np.dtype(TRIGGER_FIELDS)


def _records(rng, keys, samples, detector):
    t = np.zeros(len(keys), dtype=TRIGGER_DTYPE)
    if len(keys):
        k = np.asarray(keys)
        t["bank"], t["template_id"], t["window"] = k[:, 0], k[:, 1], k[:, 2]
        t["sample"] = samples
    t["detector"] = detector
    t["snr"] = 4.0 + rng.exponential(1.0, len(keys))
    t["snr_interp"] = t["snr"] + rng.uniform(0.0, 0.01, len(keys))
    t["dt"] = rng.uniform(-0.5, 0.5, len(keys))
    t["phase"] = rng.uniform(-np.pi, np.pi, len(keys))
    t["xi2"] = rng.exponential(1.0, len(keys))
    order = np.lexsort((t["sample"], t["template_id"], t["bank"]))
    return t[order]


def trigger_pair(seed: int, n_banks: int = 3, n_templates: int = 50, n_windows: int = 40,
                 window_len: int = 2048, rate: float = 0.1, shared: float = 0.6, spread: int = 30):
    rng = np.random.default_rng(seed)
    ka, sa, kb, sb = [], [], [], []
    for bank in range(n_banks):
        for tmpl in range(n_templates):
            for w in range(n_windows):
                lo = w * window_len
                if rng.random() < rate:
                    s = lo + int(rng.integers(0, window_len))
                    ka.append((bank, tmpl, w))
                    sa.append(s)
                    if rng.random() < shared:
                        s2 = int(np.clip(s + rng.integers(-spread, spread + 1), lo, lo + window_len - 1))
                        kb.append((bank, tmpl, w))
                        sb.append(s2)
                        continue
                if rng.random() < rate / 2:
                    kb.append((bank, tmpl, w))
                    sb.append(lo + int(rng.integers(0, window_len)))
    return _records(rng, ka, sa, 0), _records(rng, kb, sb, 1)
