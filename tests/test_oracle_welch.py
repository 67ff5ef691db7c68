"""Pins for oracle.welch (Welch PSD)."""
import numpy as np
import pytest
import scipy.signal

import oracle
from synth import coloured_noise
from synth.noise import white_noise

FS = 2048.0


def test_fft_equals_brute_dft():
    x = coloured_noise(3 * 512, seed=3)
    a = oracle.welch_psd(x, FS, nperseg=512, noverlap=256, method="fft")
    b = oracle.welch_psd(x, FS, nperseg=512, noverlap=256, method="dft")
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=0)


def test_matches_scipy_welch_same_settings():
    x = coloured_noise(32768, seed=0)
    ours = oracle.welch_psd(x, FS, 4096, 2048)
    f, ref = scipy.signal.welch(x, fs=FS, window="hann", nperseg=4096, noverlap=2048,
                                detrend=False, scaling="density", average="mean",
                                return_onesided=True, axis=-1)
    assert ours.shape == (2, 2049)
    np.testing.assert_allclose(ours, ref, rtol=1e-12, atol=0)


def test_hann_is_periodic():
    w = oracle.hann_periodic(8)
    np.testing.assert_allclose(w, [0, 0.5 - 0.5 * np.sqrt(0.5), 0.5, 0.5 + 0.5 * np.sqrt(0.5), 1,
                                   0.5 + 0.5 * np.sqrt(0.5), 0.5, 0.5 - 0.5 * np.sqrt(0.5)], atol=1e-15)


def test_windowed_parseval_identity():
    # sum_k S_k df == mean over segments of sum_n (w_n x_n)^2 / sum_n w_n^2
    rng = np.random.default_rng(5)
    x = rng.standard_normal(20000)
    L, step = 4096, 2048
    S = oracle.welch_psd(x, FS, L, L - step)
    w = oracle.hann_periodic(L)
    n_seg = (len(x) - L) // step + 1
    energy = np.mean([np.sum((w * x[s * step:s * step + L]) ** 2) for s in range(n_seg)])
    lhs = S.sum() * FS / L
    assert abs(lhs - energy / np.sum(w * w)) <= 1e-12 * abs(lhs)


def test_pure_tone_closed_form():
    # bin-centred tone a cos(2 pi k0 n / L): with a periodic Hann window all
    # power sits in bins k0 and k0 +- 1 with S = a^2 L/(3 fs) and a^2 L/(12 fs)
    L, k0, a = 4096, 300, 2.5
    n = np.arange(3 * L)
    x = a * np.cos(2 * np.pi * k0 * n / L + 0.7)
    S = oracle.welch_psd(x, FS, L, L // 2)
    assert S[k0] == pytest.approx(a * a * L / (3 * FS), rel=1e-12)
    assert S[k0 - 1] == pytest.approx(a * a * L / (12 * FS), rel=1e-12)
    assert S[k0 + 1] == pytest.approx(a * a * L / (12 * FS), rel=1e-12)
    mask = np.ones_like(S, bool)
    mask[k0 - 1:k0 + 2] = False
    assert np.max(S[mask]) < 1e-20 * S[k0]


def test_white_noise_level():
    # E[S_k] = 2 sigma^2 / fs for white noise of variance sigma^2
    sigma = 3.0
    x = white_noise(2048 * 400, sigma=sigma, seed=7, n_ch=1)
    S = oracle.welch_psd(x, FS)[0]
    level = 2 * sigma ** 2 / FS
    assert np.mean(S[1:-1]) == pytest.approx(level, rel=0.01)


def test_coloured_noise_follows_analytic_psd():
    from synth import analytic_psd
    x = coloured_noise(2048 * 256, seed=11, n_ch=1)
    S = oracle.welch_psd(x, FS)[0]
    f = np.arange(2049) * FS / 4096
    band = (f >= 20) & (f <= 1000)
    ratio = S[band] / analytic_psd(f[band])
    assert np.mean(ratio) == pytest.approx(1.0, rel=0.01)


def test_rolling_equals_slices():
    x = coloured_noise(2048 * 40, seed=2)
    R = oracle.welch_psd_rolling(x, FS, psd_len=2048 * 16, psd_hop=2048 * 8, n_psd=3)
    for j in range(3):
        np.testing.assert_array_equal(R[j], oracle.welch_psd(x[:, j * 16384: j * 16384 + 32768], FS))
