"""GPU parity: clustering into candidate events (af_cluster) and false alarm
rates (af_far) against the oracle."""
import os

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import banner, dev, need_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cluster_example.txt")


def _offsets(lens):
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def _gpu_cluster(P, x, half, off=None, max_out=None):
    xo = dev(x.astype(np.float32))
    oo = torch.from_numpy(off).cuda() if off is not None else None
    idx, val = P.cluster(xo, half, oo, max_out=max_out)
    return idx.cpu().numpy(), val.cpu().numpy()


def test_hand_worked_example():
    P = need_gpu()
    rec = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            rec[k] = [float(t) for t in v]
    x = np.array(rec["x"], dtype=np.float32)
    idx, val = _gpu_cluster(P, x, int(rec["half"][0]), np.array(rec["offsets"], dtype=np.int64))
    assert idx.tolist() == [int(v) for v in rec["candidates"]]
    np.testing.assert_array_equal(val, x[idx])


@pytest.mark.parametrize("half", [0, 1, 4, 64, 300, 1024])
def test_ragged_series_with_ties(half):
    # series shorter and longer than a 256-sample tile and than the window,
    # empty ones, and values on a coarse grid (many ties)
    P = need_gpu()
    banner(f"cluster ragged half={half}")
    rng = np.random.default_rng(half)
    lens = [0, 1, 2, 255, 256, 257, 0, 700, 3, 1500, 64]
    off = _offsets(lens)
    x = (np.round(rng.standard_normal(off[-1]) * 3) / 3).astype(np.float32)
    idx, val = _gpu_cluster(P, x, half, off)
    ref_i, ref_v = oracle.cluster(x, half, off)
    np.testing.assert_array_equal(idx, ref_i)
    np.testing.assert_array_equal(val, ref_v)


def test_single_series_edges_and_truncation():
    P = need_gpu()
    rng = np.random.default_rng(7)
    x = rng.standard_normal(5000).astype(np.float32)
    idx, _ = _gpu_cluster(P, x, 16)
    ref, _ = oracle.cluster(x, 16)
    np.testing.assert_array_equal(idx, ref)
    part, _ = _gpu_cluster(P, x, 16, max_out=10)       # the first 10 of the full list
    np.testing.assert_array_equal(part, ref[:10])
    none, _ = _gpu_cluster(P, x[:0], 16)
    assert none.size == 0
    with pytest.raises(P.AframeError, match="EINVAL"):
        _gpu_cluster(P, x, 1025)


def test_hour_scale_series_sampled():
    # 4000 (segment, slide) series of a timeslide run at 1 Hz, h = 4 s: every
    # candidate is checked by the window rule, and a sample of whole series
    # against the oracle
    P = need_gpu()
    banner("cluster 4000 series")
    rng = np.random.default_rng(11)
    lens = rng.integers(60, 4000, 4000)
    off = _offsets(lens)
    x = rng.standard_normal(off[-1]).astype(np.float32)
    idx, val = _gpu_cluster(P, x, 4, off)
    assert np.all(np.diff(idx) > 0)
    seg = np.searchsorted(off, idx, side="right") - 1
    for s in rng.choice(len(lens), 25, replace=False):
        lo, hi = off[s], off[s + 1]
        ref, _ = oracle.cluster(x[lo:hi], 4)
        np.testing.assert_array_equal(idx[seg == s] - lo, ref)
    # window rule on every candidate
    for i, s in zip(idx[::97], seg[::97]):
        lo, hi = off[s], off[s + 1]
        assert np.all(x[max(lo, i - 4):i] < x[i]) and np.all(x[i + 1:min(hi, i + 5)] <= x[i])
    np.testing.assert_array_equal(val, x[idx])


def test_far_exact():
    P = need_gpu()
    rng = np.random.default_rng(13)
    bg = np.round(rng.standard_normal(200_000), 2).astype(np.float32)   # crosses several 2^16 chunks
    q = np.concatenate([np.round(rng.standard_normal(1000), 2), [bg.min() - 1, bg.max()]]).astype(np.float32)
    T = 86400.0 * 100
    got = P.far(dev(bg), T, dev(q)).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.false_alarm_rate(bg, T, q))
    empty = P.far(dev(bg[:0]), T, dev(q)).cpu().numpy()
    assert np.all(empty == 0.0)
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.far(dev(bg), 0.0, dev(q))
