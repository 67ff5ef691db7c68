"""Pins of the clustering and false-alarm-rate oracle (oracle/events.py)."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cluster_example.txt")


def _golden():
    rec = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            key, *vals = line.split()
            rec[key] = [float(v) for v in vals]
    return rec


def test_hand_worked_example():
    g = _golden()
    idx, val = oracle.cluster(np.array(g["x"]), int(g["half"][0]), [int(v) for v in g["offsets"]])
    assert idx.tolist() == [int(v) for v in g["candidates"]]
    assert val.tolist() == [g["x"][i] for i in idx]


def _greedy(x, half, thresh):
    # independent definition: take the largest remaining sample (earliest of
    # equals), drop everything within half of it, repeat
    x = np.array(x, dtype=np.float64)
    alive = np.ones(len(x), dtype=bool)
    out = []
    while alive.any():
        i = int(np.flatnonzero(alive)[np.argmax(x[alive])])
        if x[i] <= thresh:
            break
        out.append(i)
        alive[max(0, i - half):i + half + 1] = False
    return sorted(out)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_separated_bumps_match_greedy_and_peaks(seed):
    rng = np.random.default_rng(seed)
    half, n = 8, 2000
    x = rng.uniform(0.0, 0.5, n)                        # background below the threshold 1
    peaks = np.sort(rng.choice(np.arange(20, n - 20, 2 * half + 3), 25, replace=False))
    for p in peaks:                                      # unimodal bumps, > 2 half apart
        x[p - half:p + half + 1] = np.maximum(x[p - half:p + half + 1],
                                              5.0 - np.abs(np.arange(-half, half + 1)) * 0.3)
    idx, _ = oracle.cluster(x, half)
    big = idx[x[idx] > 1.0].tolist()
    assert big == peaks.tolist()
    assert big == _greedy(x, half, 1.0)


@pytest.mark.parametrize("seed", [3, 4])
def test_window_properties_on_random_series(seed):
    rng = np.random.default_rng(seed)
    half = 5
    lens = [0, 1, 7, 40, 300]
    off = np.concatenate([[0], np.cumsum(lens)])
    x = np.round(rng.standard_normal(off[-1]) * 2) / 2     # many ties
    idx, val = oracle.cluster(x, half, off)
    for s in range(len(lens)):
        lo, hi = off[s], off[s + 1]
        mine = idx[(idx >= lo) & (idx < hi)]
        assert np.all(np.diff(mine) > half)
        for i in mine:
            w = x[max(lo, i - half):min(hi, i + half + 1)]
            assert x[i] == w.max()
            earlier = x[max(lo, i - half):i]
            assert np.all(earlier < x[i])
        if hi > lo:                                        # the series maximum's first occurrence is always kept
            assert lo + int(np.argmax(x[lo:hi])) in mine.tolist()


def test_half_zero_keeps_everything_and_plateau_keeps_first():
    x = np.array([3.0, 3.0, 3.0, 1.0])
    assert oracle.cluster(x, 0)[0].tolist() == [0, 1, 2, 3]
    assert oracle.cluster(x, 2)[0].tolist() == [0]
    assert oracle.cluster(np.array([1.0, np.nan, 2.0]), 1)[0].tolist() == []


def test_far_against_sorted_counts():
    rng = np.random.default_rng(5)
    bg = np.round(rng.standard_normal(5000), 2)
    q = np.concatenate([np.round(rng.standard_normal(300), 2), [bg.min() - 1, bg.max(), bg.max() + 1]])
    T = 3600.0 * 24
    far = oracle.false_alarm_rate(bg, T, q)
    srt = np.sort(bg)
    ref = (len(bg) - np.searchsorted(srt, q, side="right")) / T
    np.testing.assert_array_equal(far, ref)
    assert far[-3] == len(bg) / T and far[-2] == 0.0 and far[-1] == 0.0
    order = np.argsort(q)
    assert np.all(np.diff(far[order]) <= 0)
