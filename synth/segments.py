"""Lognormal science-segment layout standing in for H1-L1 coincident time.

The paper evaluates on coincident science-mode segments of O3 (Sec. IV.A).
Here 24 h is split into 40 segments whose lengths are lognormal with a median
of 30 min and sigma = sqrt(2 ln 1.2) (mean 36 min = 24 h / 40), rescaled to
sum to 24 h, clipped to [60 s, 3 h] and rounded to whole seconds; whatever the
clipping and rounding leave over goes to the longest segment.
"""
import numpy as np


def lognormal_segments(n_seg=40, total_s=86400, median_s=1800.0,
                       clip=(60, 10800), seed=0):
    rng = np.random.default_rng(seed)
    sigma = np.sqrt(2.0 * np.log(1.2))
    d = np.exp(np.log(median_s) + sigma * rng.standard_normal(n_seg))
    d *= total_s / d.sum()
    d = np.clip(np.rint(d), clip[0], clip[1]).astype(np.int64)
    d[np.argmax(d)] += total_s - int(d.sum())
    return d
