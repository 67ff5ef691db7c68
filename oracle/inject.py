"""Projection onto detectors and network SNR (oracle, test infrastructure).

* Projection (Sec. IV, signal injection): detector response
  h_d(t) = F+ h+(t - dt_d) + Fx hx(t - dt_d), F = D : e with the detector
  tensor D = (x x^T - y y^T)/2 of the arm unit vectors, the polarisation
  tensors e+ = X X^T - Y Y^T, ex = X Y^T + Y X^T of the wave's basis rotated
  by the polarisation angle psi around the source direction, and the arrival
  delay dt_d = -(r_d . s)/c of the vertex r_d against the geocentre.  Written
  from the definitions, one sample at a time (linear interpolation for the
  fractional delay, zero outside the series).
* Network SNR (footnote of Sec. I: the total SNR of the detector network):
  rho^2 = sum_d 4 df sum_{f_j >= f_low} |H_d(f_j)|^2 / S_d(f_j), H = DFT / fs,
  with S_d linearly interpolated on the PSD grid; rescaling multiplies the
  series by target / rho.

Pins (tests/test_oracle_inject.py): a detector whose arms are the wave's own
basis gives F+ = 1, Fx = 0 (and |Fx| = 1 at psi = pi/4); F+^2 + Fx^2 does not
depend on psi and F(psi + pi/2) = -F(psi); the H1-L1 delay difference never
exceeds the baseline light time (about 10 ms, Sec. IX) and reaches it along
the baseline; whole-sample delays shift exactly; the SNR of a sinusoid on a
frequency bin against a flat PSD has the closed form A^2 N / (fs S); against a
PSD given on a coarser grid, S at each sinusoid is the linear interpolation of
its two grid neighbours.
"""
import numpy as np

C_LIGHT = 299792458.0


def sky_basis(ra, dec, psi, gmst):
    """(s, X, Y): source direction and the polarisation basis, Earth-fixed."""
    phi = ra - gmst
    s = np.array([np.cos(dec) * np.cos(phi), np.cos(dec) * np.sin(phi), np.sin(dec)])
    ea = np.array([-np.sin(phi), np.cos(phi), 0.0])
    ed = np.array([-np.sin(dec) * np.cos(phi), -np.sin(dec) * np.sin(phi), np.cos(dec)])
    X = np.cos(psi) * ea + np.sin(psi) * ed
    Y = -np.sin(psi) * ea + np.cos(psi) * ed
    return s, X, Y


def antenna(det_row, ra, dec, psi, gmst):
    """(F+, Fx, dt) of one detector row [vertex, x arm, y arm]."""
    r, x, y = det_row[:3], det_row[3:6], det_row[6:9]
    s, X, Y = sky_basis(ra, dec, psi, gmst)
    D = 0.5 * (np.outer(x, x) - np.outer(y, y))
    fp = np.sum(D * (np.outer(X, X) - np.outer(Y, Y)))
    fx = np.sum(D * (np.outer(X, Y) + np.outer(Y, X)))
    return fp, fx, -np.dot(r, s) / C_LIGHT


def project(hp, hc, sky, det, fs):
    """hp, hc [n_inj, len]; sky [n_inj, 4]; det [n_det, 9] -> [n_inj, n_det, len]."""
    hp = np.asarray(hp, dtype=np.float64)
    hc = np.asarray(hc, dtype=np.float64)
    n_inj, n = hp.shape
    out = np.zeros((n_inj, len(det), n))
    for i in range(n_inj):
        for d in range(len(det)):
            fp, fx, dt = antenna(det[d], *sky[i])
            for k in range(n):
                u = k - dt * fs
                i0 = int(np.floor(u))
                w = u - i0
                val = lambda h, j: h[j] if 0 <= j < n else 0.0
                a_p = (1 - w) * val(hp[i], i0) + w * val(hp[i], i0 + 1)
                a_c = (1 - w) * val(hc[i], i0) + w * val(hc[i], i0 + 1)
                out[i, d, k] = fp * a_p + fx * a_c
    return out


def network_snr(sig, psd, df, fs, f_low):
    """sig [n_inj, n_det, len]; psd [n_det, n_freq] on the grid m*df -> [n_inj]."""
    sig = np.asarray(sig, dtype=np.float64)
    n = sig.shape[-1]
    f = np.arange(n // 2) * fs / n
    grid = np.arange(psd.shape[-1]) * df
    rho2 = np.zeros(sig.shape[0])
    for d in range(sig.shape[1]):
        S = np.interp(f, grid, psd[d])
        use = (f >= f_low) & (f < grid[-1]) & (S > 0)
        H = np.fft.fft(sig[:, d, :], axis=-1)[:, :n // 2] / fs
        rho2 += 4.0 * (fs / n) * np.sum(np.abs(H[:, use]) ** 2 / S[use], axis=-1)
    return np.sqrt(rho2)
