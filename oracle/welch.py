"""Welch power spectral density (oracle, FP64).

The paper estimates the noise PSD from a background stretch that precedes the
data being whitened: 8 s in training (Sec. IV.B, noise sampling) and the first
64 s of the snapshotter state at inference (Sec. VI).  It does not state the
estimator's parameters; the reading used throughout is Welch's method with
2 s periodic-Hann segments at 50 % overlap, mean (not median) averaging, no
detrending and one-sided density scaling:

    w_n  = 1/2 - 1/2 cos(2 pi n / L),           n = 0 .. L-1
    P_s(k) = | sum_n w_n x[s*step + n] e^{-2 pi i k n / L} |^2
    S_k  = c_k * mean_s P_s(k) / (fs * sum_n w_n^2),  c_0 = c_{L/2} = 1, else 2.

Pins (tests/test_oracle_welch.py): FFT path == brute-force DFT; equality with
scipy.signal.welch under the same settings; the windowed-Parseval identity
sum_k S_k df = mean_s sum_n (w_n x_n)^2 / sum w^2; a pure tone's peak bin; and
E[S] = 2 sigma^2 / fs for white noise.
"""
import numpy as np


def hann_periodic(L):
    n = np.arange(L, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / L)


def _segments(x, nperseg, noverlap):
    step = nperseg - noverlap
    n_seg = (x.shape[-1] - nperseg) // step + 1
    if n_seg < 1:
        raise ValueError("input shorter than one Welch segment")
    starts = step * np.arange(n_seg)
    return np.stack([x[..., s:s + nperseg] for s in starts], axis=-2)  # [..., n_seg, L]


def periodogram_dft(seg):
    """|DFT|^2 of each row of `seg` by the O(L^2) definition (small L only)."""
    L = seg.shape[-1]
    k = np.arange(L // 2 + 1)[:, None]
    n = np.arange(L)[None, :]
    E = np.exp(-2j * np.pi * ((k * n) % L) / L)
    X = seg @ E.T
    return np.abs(X) ** 2


def welch_psd(x, fs, nperseg=4096, noverlap=2048, method="fft"):
    """One-sided Welch PSD of x [..., n] -> [..., nperseg//2 + 1] (float64)."""
    x = np.asarray(x, dtype=np.float64)
    w = hann_periodic(nperseg)
    segs = _segments(x, nperseg, noverlap) * w
    if method == "fft":
        P = np.abs(np.fft.rfft(segs, axis=-1)) ** 2
    elif method == "dft":
        P = periodogram_dft(segs)
    else:
        raise ValueError(method)
    S = P.mean(axis=-2) / (fs * np.sum(w * w))
    c = np.full(S.shape[-1], 2.0)
    c[0] = 1.0
    if nperseg % 2 == 0:
        c[-1] = 1.0
    return S * c


def welch_psd_rolling(x, fs, psd_len, psd_hop, n_psd, nperseg=4096, noverlap=2048):
    """PSD_j = welch_psd(x[..., j*psd_hop : j*psd_hop + psd_len]) for j < n_psd.

    Returns [n_psd, ..., nperseg//2 + 1].  This is the rolling background of
    the inference stage: each hop of whitened output uses the PSD of the
    `psd_len` samples that precede it.
    """
    return np.stack([welch_psd(x[..., j * psd_hop: j * psd_hop + psd_len], fs, nperseg, noverlap)
                     for j in range(n_psd)])
