"""Inverse-ASD whitening filter and time-domain whitening (oracle, FP64).

The paper builds a whitening filter from the background PSD, whitens in the
frequency domain, transforms back and removes 0.5 s at each edge that the
filter's settle-in corrupts (Sec. IV.B noise sampling; Sec. VI; Table III).
Read as a finite impulse response of 1 s total length (0.5 s per side):

    A_k   = 1/sqrt(S_k) for f_k = k fs / L >= f_hp (and S_k > 0), else 0
    q     = irfft_L(A)                       (real, even, zero phase)
    h[m]  = q[m mod L] * (1 + cos(pi m / M)) / 2  for |m| < M, M = fduration fs / 2
    y[n]  = sqrt(2 / fs) * sum_m h[m] x[n - m]   for M <= n < N - M

The sqrt(2/fs) factor maps a one-sided PSD S to unit variance per unit
bandwidth: white noise of variance s^2 (S = 2 s^2 / fs) comes out with unit
variance, and Gaussian noise with the filter's own PSD comes out with variance
equal to the pass-band fraction (1 - 2 f_hp / fs).  With a rolling PSD the
output sample n uses the filter of the hop that contains it.

Pins (tests/test_oracle_whiten.py): white noise -> x / sigma exactly; the
exact inverse for an ASD whose inverse is a short cosine sum (noise coloured by
the exact inverse of the resulting filter comes back as sqrt(2/fs) times the
white input at every output sample); taps equal the written-out cosine sum;
output variance equal to the band fraction; scale invariance; direct sum ==
FFT convolution == per-sample dot products.
"""
import numpy as np
import scipy.signal


def whitening_fir(psd, fs, highpass=32.0, fduration=1.0):
    """psd [..., L/2+1] -> taps [..., 2M-1] with taps[..., m + M - 1] = h[m]."""
    psd = np.asarray(psd, dtype=np.float64)
    F = psd.shape[-1]
    L = 2 * (F - 1)
    f = np.arange(F) * fs / L
    with np.errstate(divide="ignore"):
        A = np.where((f >= highpass) & (psd > 0), 1.0 / np.sqrt(np.where(psd > 0, psd, 1.0)), 0.0)
    q = np.fft.irfft(A, n=L, axis=-1)
    M = int(round(fduration * fs / 2))
    if 2 * M - 1 > L:
        raise ValueError("filter longer than the PSD's segment length")
    m = np.arange(-(M - 1), M)
    taper = 0.5 * (1.0 + np.cos(np.pi * m / M))
    return q[..., m % L] * taper


def _conv_valid(x, taps, method):
    if method == "direct":
        return np.convolve(x, taps, mode="valid")
    if method == "fft":
        return scipy.signal.oaconvolve(x, taps, mode="valid")
    raise ValueError(method)


def whiten(x, psd, fs, highpass=32.0, fduration=1.0, method="direct"):
    """x [n_ch, N], psd [n_ch, F] -> y [n_ch, N - 2M] (output n = M .. N-M-1)."""
    x = np.asarray(x, dtype=np.float64)
    taps = whitening_fir(psd, fs, highpass, fduration)
    M = (taps.shape[-1] + 1) // 2
    N = x.shape[-1]
    out = np.empty((x.shape[0], N - 2 * M))
    for c in range(x.shape[0]):
        full = _conv_valid(x[c], taps[c], method)  # sample n = i + M - 1, i = 0 .. N-2M+1
        out[c] = full[1:N - 2 * M + 1]
    return out * np.sqrt(2.0 / fs)


def whiten_piecewise(x, psds, fs, n0, n_out, psd_hop, highpass=32.0, fduration=1.0,
                     method="fft"):
    """Whitened output y[c, i] for raw sample n0 + i, i < n_out, using the
    filter of hop j = min(i // psd_hop, n_psd - 1); psds is [n_psd, n_ch, F]."""
    x = np.asarray(x, dtype=np.float64)
    taps = whitening_fir(psds, fs, highpass, fduration)   # [n_psd, n_ch, 2M-1]
    M = (taps.shape[-1] + 1) // 2
    n_psd = taps.shape[0]
    if n0 < M or n0 + n_out + M > x.shape[-1]:
        raise ValueError("output range needs M samples of context on each side")
    y = np.empty((x.shape[0], n_out))
    for j in range(n_psd):
        lo = j * psd_hop
        hi = n_out if j == n_psd - 1 else min((j + 1) * psd_hop, n_out)
        if hi <= lo:
            continue
        for c in range(x.shape[0]):
            seg = x[c, n0 + lo - (M - 1): n0 + hi + (M - 1)]
            y[c, lo:hi] = _conv_valid(seg, taps[j, c], method)
    return y * np.sqrt(2.0 / fs)


def whiten_at(x, taps, positions, fs):
    """sqrt(2/fs) * sum_m h[m] x[n - m] at raw sample positions n (1-D x, taps)."""
    M = (len(taps) + 1) // 2
    pos = np.asarray(positions)
    idx = pos[:, None] + np.arange(M - 1, -M, -1)[None, :]   # n - m for m = -(M-1)..M-1
    return (x[idx] @ taps) * np.sqrt(2.0 / fs)
