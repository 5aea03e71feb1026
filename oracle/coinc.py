"""Coincidence of two detectors' triggers (test infrastructure only).

Sec. II.A passes the triggers to a coincidence generator that pairs the
triggers of the same template within the light travel time between the
detectors; the triggers in no pair, from times when several detectors
observe, form the background.  Restated as a plain definition: every pair
(i, j) of the two lists with the same bank and template whose peak samples
differ by at most max_dt samples (inclusive), in order of i, then j.  Each
pair carries the network SNR sqrt(snr_a^2 + snr_b^2) and the arrival
difference (sample_b + dt_b) - (sample_a + dt_a) in samples, with each
trigger's sub-sample refinement.

This is the definition written out as a double loop over both lists, for
the small lists the tests use.
"""

from __future__ import annotations

import math


def coincidences(a, b, max_dt: int):
    """a, b: sequences of records with fields bank, template_id, sample, snr, dt
    (numpy structured arrays work).  Returns (pairs, background): pairs is a
    list of (i, j, bank, template_id, snr_net, dt) in order of i, then j;
    background is a list of len(a) + len(b) flags, 1 for a trigger in no pair."""
    pairs = []
    used_b = [False] * len(b)
    bg_a = []
    for i in range(len(a)):
        x = a[i]
        found = False
        for j in range(len(b)):
            y = b[j]
            if int(x["bank"]) != int(y["bank"]) or int(x["template_id"]) != int(y["template_id"]):
                continue
            if abs(int(x["sample"]) - int(y["sample"])) > max_dt:
                continue
            snr_net = math.sqrt(float(x["snr"]) ** 2 + float(y["snr"]) ** 2)
            dt = (int(y["sample"]) - int(x["sample"])) + (float(y["dt"]) - float(x["dt"]))
            pairs.append((i, j, int(x["bank"]), int(x["template_id"]), snr_net, dt))
            used_b[j] = True
            found = True
        bg_a.append(0 if found else 1)
    return pairs, bg_a + [0 if u else 1 for u in used_b]
