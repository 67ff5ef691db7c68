"""Sanity checks of the seeded input generators (not part of the method)."""
import numpy as np

from synth import lognormal_segments, inject_chirps, newtonian_chirp, coloured_noise
from synth.chirps import _snr2


def test_segments_layout():
    d = lognormal_segments(seed=0)
    assert len(d) == 40 and d.sum() == 86400
    assert d.min() >= 60
    assert np.all(d == np.round(d))


def test_chirp_frequency_sweeps_up():
    h, n_after = newtonian_chirp(30.0)
    assert len(h) > 2048 * 0.5 and n_after >= 0
    zc = np.nonzero(np.diff(np.signbit(h)))[0]
    gaps = np.diff(zc)
    assert gaps[:20].mean() > gaps[-20:].mean()      # zero crossings get denser


def test_injection_hits_target_snr():
    x = np.zeros((2, 2048 * 130))
    inj = inject_chirps(x, seed=1)
    assert len(inj) == 2
    for rec in inj:
        tc = rec["tc"]
        seg = x[:, tc - 2048 * 30: tc + 2048]
        rho = np.sqrt(sum(_snr2(seg[c], 2048.0) for c in range(2)))
        assert abs(rho - rec["snr"]) < 0.02 * rec["snr"]


def test_noise_is_seeded():
    a = coloured_noise(4096, seed=3)
    b = coloured_noise(4096, seed=3)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a[0], a[1])
