"""Pins of the projection and network-SNR oracle (oracle/inject.py)."""
import numpy as np
import pytest

import oracle
from oracle.inject import sky_basis
from synth.detectors import ligo_detectors, sky_draws

FS = 2048.0


def test_detector_aligned_with_the_wave_basis():
    # arms along the wave's own basis vectors: F+ = 1, Fx = 0 at psi = 0 and
    # F+ = 0, |Fx| = 1 at psi = pi/4 (the tensor contractions written out)
    ra, dec, gmst = 1.1, -0.4, 0.3
    _, X, Y = sky_basis(ra, dec, 0.0, gmst)
    row = np.concatenate([[0.0, 0.0, 0.0], X, Y])
    fp, fx, dt = oracle.antenna(row, ra, dec, 0.0, gmst)
    assert fp == pytest.approx(1.0, abs=1e-14) and fx == pytest.approx(0.0, abs=1e-14) and dt == 0.0
    fp, fx, _ = oracle.antenna(row, ra, dec, np.pi / 4, gmst)
    assert fp == pytest.approx(0.0, abs=1e-14) and abs(fx) == pytest.approx(1.0, abs=1e-14)


def test_polarisation_rotation_properties():
    det = ligo_detectors()
    for ra, dec, psi, gmst in sky_draws(20, seed=1):
        for row in det:
            fp, fx, dt = oracle.antenna(row, ra, dec, psi, gmst)
            fp2, fx2, dt2 = oracle.antenna(row, ra, dec, psi + 0.7, gmst)
            assert fp ** 2 + fx ** 2 == pytest.approx(fp2 ** 2 + fx2 ** 2, rel=1e-12)
            fp3, fx3, _ = oracle.antenna(row, ra, dec, psi + np.pi / 2, gmst)
            assert fp3 == pytest.approx(-fp, abs=1e-12) and fx3 == pytest.approx(-fx, abs=1e-12)
            assert dt == dt2 and fp ** 2 + fx ** 2 <= 1.0 + 1e-12


def test_delay_bounded_by_the_baseline_light_time():
    # about 10 ms for the two LIGO sites (Sec. IX); reached along the baseline
    det = ligo_detectors()
    base = det[1, :3] - det[0, :3]
    t_light = np.linalg.norm(base) / oracle.inject.C_LIGHT
    assert 9.9e-3 < t_light < 10.1e-3
    for ra, dec, psi, gmst in sky_draws(200, seed=2):
        d = oracle.antenna(det[1], ra, dec, psi, gmst)[2] - oracle.antenna(det[0], ra, dec, psi, gmst)[2]
        assert abs(d) <= t_light * (1 + 1e-12)
    u = base / np.linalg.norm(base)                      # source along the baseline (gmst 0)
    ra, dec = np.arctan2(u[1], u[0]), np.arcsin(u[2])
    d = oracle.antenna(det[1], ra, dec, 0.0, 0.0)[2] - oracle.antenna(det[0], ra, dec, 0.0, 0.0)[2]
    assert d == pytest.approx(-t_light, rel=1e-12)


def test_whole_sample_delay_shifts_exactly():
    rng = np.random.default_rng(3)
    hp, hc = rng.standard_normal((2, 1, 64))
    row = np.concatenate([[0.0, 0.0, 0.0], [1.0, 0, 0], [0, 1.0, 0]])
    ra, dec, psi, gmst = 0.0, np.pi / 2, 0.0, 0.0        # overhead of the xy plane
    fp, fx, _ = oracle.antenna(row, ra, dec, psi, gmst)
    row[:3] = -3.0 / FS * oracle.inject.C_LIGHT * np.array([0, 0, 1.0])   # dt = +3 samples
    out = oracle.project(hp, hc, np.array([[ra, dec, psi, gmst]]), row[None, :], FS)[0, 0]
    ref = np.zeros(64)
    ref[3:] = fp * hp[0, :61] + fx * hc[0, :61]
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


def test_snr_of_a_sinusoid_on_a_bin():
    n, m, A, S0 = 4096, 300, 2.5, 4e-3
    t = np.arange(n) / FS
    sig = np.zeros((1, 2, n))
    sig[0, 0] = A * np.cos(2 * np.pi * m * FS / n * t)
    psd = np.full((2, 4097), S0)
    rho = oracle.network_snr(sig, psd, FS / 8192, FS, 20.0)[0]
    assert rho == pytest.approx(np.sqrt(A * A * n / (FS * S0)), rel=1e-12)
    sig[0, 1] = sig[0, 0]                                    # two detectors: quadrature sum
    rho2 = oracle.network_snr(sig, psd, FS / 8192, FS, 20.0)[0]
    assert rho2 == pytest.approx(np.sqrt(2) * rho, rel=1e-12)
    assert oracle.network_snr(sig, psd, FS / 8192, FS, m * FS / n + 1)[0] < 1e-9 * rho   # below f_low


def test_snr_interpolates_a_non_flat_psd_linearly():
    # PSD given every 1.5 Hz with unrelated values per grid point; sinusoids on
    # the 0.5 Hz bins of a 2 s series at 150.5 Hz and 302 Hz fall one third of
    # the way from a grid point to the next, so S there is (2/3) S_k + (1/3) S_k+1,
    # and one at 301.5 Hz falls on grid point 201.  Each contributes A^2 N / (fs S)
    # to rho^2.  Nearest-grid, swapped-weight or shifted-index readings all differ.
    n, df = 4096, 1.5
    rng = np.random.default_rng(7)
    psd = rng.uniform(1e-3, 3e-3, (2, 700))
    t = np.arange(n) / FS
    sig = np.zeros((1, 2, n))
    amps = {(0, 301): 1.3, (0, 604): 0.7, (1, 603): 2.1}
    for (d, m), a in amps.items():
        sig[0, d] += a * np.cos(2 * np.pi * m * FS / n * t)
    s1 = (2 * psd[0, 100] + psd[0, 101]) / 3            # 150.5 Hz between 150.0 and 151.5
    s2 = (2 * psd[0, 201] + psd[0, 202]) / 3            # 302.0 Hz between 301.5 and 303.0
    s3 = psd[1, 201]                                    # 301.5 Hz on the grid
    rho2 = n / FS * (1.3 ** 2 / s1 + 0.7 ** 2 / s2 + 2.1 ** 2 / s3)
    assert oracle.network_snr(sig, psd, df, FS, 20.0)[0] == pytest.approx(np.sqrt(rho2), rel=1e-10)
