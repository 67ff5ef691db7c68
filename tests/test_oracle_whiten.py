"""Pins for oracle.whiten (inverse-ASD FIR and whitening)."""
import numpy as np
import pytest

import oracle
from synth import analytic_psd, coloured_noise
from synth.noise import white_noise

FS = 2048.0
F = 2049
f_grid = np.arange(F) * FS / 4096


def test_flat_psd_without_highpass_is_division_by_sigma():
    # flat PSD 2 sigma^2/fs -> A constant -> q a scaled delta -> y = x / sigma
    sigma = 0.37
    x = white_noise(8192, sigma=sigma, seed=1)
    psd = np.full((2, F), 2 * sigma ** 2 / FS)
    y = oracle.whiten(x, psd, FS, highpass=0.0)
    np.testing.assert_allclose(y, x[:, 1024:-1024] / sigma, rtol=0, atol=1e-12)


def test_fir_matches_cosine_sum_definition():
    # h[m] = taper(m) * (1/L) sum_k c_k A_k cos(2 pi k m / L), written out
    rng = np.random.default_rng(4)
    psd = rng.uniform(0.5, 2.0, F)
    h = oracle.whitening_fir(psd, FS, highpass=32.0)
    L, M = 4096, 1024
    A = np.where(f_grid >= 32.0, 1 / np.sqrt(psd), 0.0)
    c = np.full(F, 2.0)
    c[0] = c[-1] = 1.0
    for m in [0, 1, 5, 100, 777, 1023, -1023, -40]:
        k = np.arange(F)
        q = np.sum(c * A * np.cos(2 * np.pi * k * m / L)) / L
        taper = 0.5 * (1 + np.cos(np.pi * m / M))
        assert h[m + M - 1] == pytest.approx(q * taper, rel=1e-9, abs=1e-15)
    assert h.shape == (2047,)
    np.testing.assert_allclose(h, h[::-1], rtol=0, atol=1e-15)   # zero phase


def test_band_fraction_variance():
    # coloured noise whitened with its own PSD: unit PSD in band -> variance
    # = (fs/2 - f_hp) / (fs/2) = 0.96875 (minus a small truncation loss)
    x = coloured_noise(2048 * 512, seed=21)
    psd = np.broadcast_to(analytic_psd(f_grid), (2, F))
    y = oracle.whiten(x, psd, FS, method="fft")
    v = y.var(axis=1)
    np.testing.assert_allclose(v, 0.96875, rtol=0.012)


def test_fir_response_tracks_inverse_asd():
    # the tapered 1 s FIR's frequency response follows 1/sqrt(S) wherever S is
    # smooth on the ~1 Hz scale of the taper: this pins the irfft scaling and
    # the placement of the taper around m = 0
    S = analytic_psd(f_grid)
    h = oracle.whitening_fir(S, FS, highpass=32.0)
    m = np.arange(-1023, 1024)
    f = f_grid[(f_grid >= 48) & (f_grid <= 1000)]
    H = np.cos(2 * np.pi * np.outer(f, m) / FS) @ h
    np.testing.assert_allclose(H * np.sqrt(analytic_psd(f)), 1.0, rtol=2e-3)


def test_scale_invariance():
    x = coloured_noise(16384, seed=5)
    psd = oracle.welch_psd(x, FS)
    y1 = oracle.whiten(x, psd, FS)
    y2 = oracle.whiten(1e21 * x, 1e42 * psd, FS)
    np.testing.assert_allclose(y2, y1, rtol=1e-10, atol=1e-12)


def test_direct_fft_and_pointwise_agree():
    x = coloured_noise(12000, seed=6)
    psd = oracle.welch_psd(x, FS)
    yd = oracle.whiten(x, psd, FS, method="direct")
    yf = oracle.whiten(x, psd, FS, method="fft")
    np.testing.assert_allclose(yf, yd, atol=1e-9 * np.abs(yd).max())
    taps = oracle.whitening_fir(psd, FS)
    pos = np.array([1024, 5000, 12000 - 1025])
    for c in range(2):
        np.testing.assert_allclose(oracle.whiten_at(x[c], taps[c], pos, FS), yd[c, pos - 1024],
                                   rtol=1e-10, atol=1e-12)


def test_piecewise_single_hop_equals_plain_and_hops_switch():
    x = coloured_noise(2048 * 24, seed=8)
    psd = oracle.welch_psd(x, FS)
    n = x.shape[1]
    y = oracle.whiten(x, psd, FS)
    yp = oracle.whiten_piecewise(x, psd[None], FS, n0=1024, n_out=n - 2048, psd_hop=10 ** 9)
    np.testing.assert_allclose(yp, y, atol=1e-9)
    psd2 = np.stack([psd, 4 * psd])          # hop 1 uses a PSD 4x larger -> output halves
    yq = oracle.whiten_piecewise(x, psd2, FS, n0=1024, n_out=n - 2048, psd_hop=16384)
    np.testing.assert_allclose(yq[:, :16384], y[:, :16384], atol=1e-9)
    np.testing.assert_allclose(yq[:, 16384:], 0.5 * y[:, 16384:], atol=1e-9)


def test_exact_inverse_of_a_short_cosine_sum_asd():
    # An inverse ASD A(f) = a + 2 b1 cos(2 pi f/fs) + 2 b5 cos(10 pi f/fs) has the
    # impulse response q[0] = a, q[+-1] = b1, q[+-5] = b5 and nothing else, so the
    # truncated filter is h[0] = a, h[+-1] = b1 t(1), h[+-5] = b5 t(5) with the
    # taper t(m) = (1 + cos(pi m / M)) / 2.  Noise coloured by the exact inverse
    # of that filter (division by its transfer function on a periodic grid) is
    # whitened back to sqrt(2/fs) times the white input at every output sample.
    fs, L, N = 2048.0, 4096, 1 << 15
    a, b1, b5 = 1.0, 0.2, -0.15
    M = 1024
    t = lambda m: 0.5 * (1.0 + np.cos(np.pi * m / M))
    f = np.arange(L // 2 + 1) * fs / L
    A = a + 2 * b1 * np.cos(2 * np.pi * f / fs) + 2 * b5 * np.cos(10 * np.pi * f / fs)
    psd = np.tile(1.0 / A ** 2, (2, 1))
    z = np.random.default_rng(11).standard_normal((2, N))
    w = 2 * np.pi * np.arange(N // 2 + 1) / N
    G = a + 2 * b1 * t(1) * np.cos(w) + 2 * b5 * t(5) * np.cos(5 * w)
    x = np.fft.irfft(np.fft.rfft(z, axis=-1) / G, n=N, axis=-1)
    y = oracle.whiten(x, psd, fs, highpass=0.0, fduration=1.0)
    np.testing.assert_allclose(y, np.sqrt(2.0 / fs) * z[:, M:N - M], rtol=0, atol=1e-12)
