"""Detector geometry and injection parameters (inputs, not method).

The two LIGO detectors as a table of vertex positions (metres, Earth-centred
Earth-fixed) and arm unit vectors, built from their published geodetic
vertex coordinates and arm azimuths (measured clockwise from north, arms
taken horizontal) on the WGS-84 ellipsoid.  Also seeded sky positions and
polarisation pairs for injection campaigns.
"""
import numpy as np

from .chirps import _hilbert_mask, newtonian_chirp

# name: latitude (deg N), longitude (deg E), height (m), x-arm and y-arm azimuths (deg)
SITES = {
    "H1": (46.455147, -119.407657, 142.554, 324.0006, 234.0006),
    "L1": (30.562894, -90.774240, -6.574, 252.2835, 162.2835),
}
_A, _F = 6378137.0, 1.0 / 298.257223563   # WGS-84


def detector_row(lat_deg, lon_deg, h, az_x, az_y):
    """[vertex xyz, x-arm unit xyz, y-arm unit xyz] in Earth-fixed coordinates."""
    phi, lam = np.radians(lat_deg), np.radians(lon_deg)
    e2 = _F * (2.0 - _F)
    nrad = _A / np.sqrt(1.0 - e2 * np.sin(phi) ** 2)
    r = np.array([(nrad + h) * np.cos(phi) * np.cos(lam), (nrad + h) * np.cos(phi) * np.sin(lam),
                  (nrad * (1.0 - e2) + h) * np.sin(phi)])
    east = np.array([-np.sin(lam), np.cos(lam), 0.0])
    north = np.array([-np.sin(phi) * np.cos(lam), -np.sin(phi) * np.sin(lam), np.cos(phi)])
    arm = lambda az: np.cos(np.radians(az)) * north + np.sin(np.radians(az)) * east
    return np.concatenate([r, arm(az_x), arm(az_y)])


def ligo_detectors():
    """float64 [2, 9]: H1 then L1."""
    return np.stack([detector_row(*SITES[k]) for k in ("H1", "L1")])


def sky_draws(n, seed=0):
    """float64 [n, 4]: ra uniform, dec with uniform sin(dec), psi uniform in
    [0, pi), gmst uniform (an isotropic population at random sidereal times)."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0, 2 * np.pi, n), np.arcsin(rng.uniform(-1, 1, n)),
                     rng.uniform(0, np.pi, n), rng.uniform(0, 2 * np.pi, n)], axis=1)


def polarisation_pairs(n, length, fs=2048.0, seed=0, mchirp=(20.0, 40.0), f_low=30.0):
    """float32 [n, length] twice: a Newtonian chirp as h+ and its quadrature
    as hx, ending 0.25 s before the end of the window."""
    rng = np.random.default_rng(seed)
    hp = np.zeros((n, length), dtype=np.float64)
    hc = np.zeros((n, length), dtype=np.float64)
    for i in range(n):
        h, _ = newtonian_chirp(rng.uniform(*mchirp), fs=fs, f_low=f_low)
        h = h[-(length - int(0.25 * fs)):]
        a = np.fft.ifft(np.fft.fft(h) * _hilbert_mask(len(h)))
        e = length - int(0.25 * fs)
        hp[i, e - len(h):e] = a.real
        hc[i, e - len(h):e] = a.imag
    return hp.astype(np.float32), hc.astype(np.float32)
