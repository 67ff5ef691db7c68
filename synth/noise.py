"""Gaussian noise coloured by an analytic detector PSD.

The paper analyses LIGO O3 strain resampled to 2048 Hz (Sec. IV.A); that data
is not available here, so stationary Gaussian noise with the analytic one-sided
PSD S(f) = 1e-46 [(f/30)^-4 + 1 + (f/300)^2] 1/Hz stands in for it.  Below
`f_floor` (10 Hz) the PSD is held flat at S(f_floor) and the DC bin is zero, so
the sub-band power that the 32 Hz high-pass later removes stays within a
factor ~80 of the in-band power.
"""
import numpy as np

FS = 2048.0


def analytic_psd(f, f_floor=10.0, scale=1e-46):
    """One-sided PSD S(f) in 1/Hz with a flat floor below `f_floor`.

    f_floor=None disables the floor (used only by stress tests); f=0 returns 0.
    """
    f = np.asarray(f, dtype=np.float64)
    fe = f if f_floor is None else np.maximum(f, f_floor)
    with np.errstate(divide="ignore"):
        s = scale * ((fe / 30.0) ** -4 + 1.0 + (fe / 300.0) ** 2)
    return np.where(f > 0, s, 0.0)


def coloured_noise(n, fs=FS, seed=0, n_ch=2, f_floor=10.0, rng=None):
    """Return float64 array [n_ch, n] of noise with one-sided PSD `analytic_psd`.

    Frequency-domain colouring of one length-n block per channel: the rfft bin
    k gets sqrt(S_k n fs / 4) (g1 + i g2) with g1, g2 standard normal, so that
    E|X_k|^2 = n fs S_k / 2 (one-sided density convention); the Nyquist bin of
    an even n is real with variance n fs S_k / 2.  Channels are independent.
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    nf = n // 2 + 1
    f = np.arange(nf) * (fs / n)
    s = analytic_psd(f, f_floor=f_floor)
    out = np.empty((n_ch, n), dtype=np.float64)
    for c in range(n_ch):
        g = rng.standard_normal((2, nf))
        amp = np.sqrt(s * n * fs / 4.0)
        spec = amp * (g[0] + 1j * g[1])
        if n % 2 == 0:
            spec[-1] = np.sqrt(s[-1] * n * fs / 2.0) * g[0, -1]
        spec[0] = 0.0
        out[c] = np.fft.irfft(spec, n=n)
    return out


def white_noise(n, sigma=1.0, seed=0, n_ch=2):
    """Float64 [n_ch, n] white Gaussian noise of standard deviation sigma."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal((n_ch, n))
