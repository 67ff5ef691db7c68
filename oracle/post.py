"""Windowing, integration and rank agreement (oracle, FP64).

* Windows (Sec. II, Sec. VI): window i of the whitened series covers samples
  [i*stride, i*stride + window) of every detector; with n samples there are
  floor((n - window) / stride) + 1 windows.  The paper uses a 4 Hz inference
  rate (stride fs/4); the workloads here use 16 Hz (stride 128) or 1 Hz.
* Integration (Sec. II; Table III): the predictions are smoothed with a 1 s
  top hat.  Read as a causal, right-aligned mean over W = rate * 1 s
  consecutive predictions, valid mode:  I_i = (1/W) sum_{j=i}^{i+W-1} p_j,
  i = 0 .. n - W, attributed to the time of prediction i + W - 1.
* Kendall's tau-b over pairs (for rank agreement between two statistics),
  by the O(n^2) definition.

Pins (tests/test_oracle_post.py): integrate == cumulative-sum difference ==
numpy.convolve(valid); tau-b == scipy.stats.kendalltau on random and tied data;
window count and content against a brute-force slice.
"""
import numpy as np


def n_windows(n, window, stride):
    return 0 if n < window else (n - window) // stride + 1


def unfold_windows(y, window, stride, shifts=None, wrap=0):
    """y [n_ch, n] -> [n_w, n_ch, window]; channel c of window i starts at
    i*stride + shifts[c] (taken modulo `wrap` sample by sample when wrap > 0)."""
    n_ch, n = y.shape
    if shifts is None:
        shifts = np.zeros(n_ch, dtype=np.int64)
    nw = n_windows(n, window, stride)
    out = np.empty((nw, n_ch, window), dtype=y.dtype)
    t = np.arange(window)
    for i in range(nw):
        for c in range(n_ch):
            idx = i * stride + shifts[c] + t
            if wrap > 0:
                idx = idx % wrap
            out[i, c] = y[c, idx]
    return out


def integrate(p, width):
    p = np.asarray(p, dtype=np.float64)
    n = len(p)
    if n < width:
        return np.zeros(0)
    return np.array([p[i:i + width].sum() for i in range(n - width + 1)]) / width


def kendall_tau_b(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(a)
    if n < 2:
        return np.nan
    da = np.sign(a[:, None] - a[None, :])
    db = np.sign(b[:, None] - b[None, :])
    iu = np.triu_indices(n, 1)
    s = (da * db)[iu].sum()
    n0 = n * (n - 1) / 2
    n1 = n0 - np.count_nonzero(da[iu])      # pairs tied in a
    n2 = n0 - np.count_nonzero(db[iu])      # pairs tied in b
    return s / np.sqrt((n0 - n1) * (n0 - n2))
