"""Candidate events and false alarm rates (oracle, test infrastructure).

* Clustering (Sec. II): the integrated series is clustered so that one event
  gives one trigger, and the largest integrated value over an 8 s window is
  the event's detection statistic.  Read as a local-maximum rule with a
  half-window of h samples (4 s at the statistic's rate): sample i of a series
  is a candidate iff x[i] > x[j] for every j in [i - h, i) and x[i] >= x[j]
  for every j in (i, i + h], j within the series.  Written below as that
  definition, sample by sample.
* False alarm rate (Sec. IX): background events with a statistic greater
  than x, divided by the livetime of the background (timeslides).

Pins (tests/test_oracle_events.py): a hand-worked example stored under
tests/golden/ with its derivation; on series of separated bumps the rule picks
exactly the bump peaks and agrees with an independent greedy suppression
(take the global maximum, remove everything within h, repeat); candidates are
more than h apart and each is the maximum of its window; equal values resolve
to the earliest.  FAR equals a sort-and-search count, is non-increasing in x,
is n_bg / livetime below every background value and 0 at the largest.
"""
import numpy as np


def cluster(x, half, offsets=None):
    """Candidates of x [n] (float); series s is x[offsets[s]:offsets[s+1]]
    (one series when offsets is None).  Returns (indices int64, values)."""
    x = np.asarray(x)
    n = len(x)
    if offsets is None:
        offsets = [0, n]
    idx = []
    for s in range(len(offsets) - 1):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        for i in range(lo, hi):
            left = x[max(i - half, lo):i]
            right = x[i + 1:min(i + half, hi - 1) + 1]
            if np.all(left < x[i]) and np.all(right <= x[i]):
                idx.append(i)
    idx = np.array(idx, dtype=np.int64)
    return idx, x[idx]


def false_alarm_rate(bg, livetime, x):
    """#{background statistics > x} / livetime for each query in x (FP64)."""
    bg = np.asarray(bg)
    return np.array([np.count_nonzero(bg > q) for q in np.asarray(x)], dtype=np.float64) / float(livetime)
