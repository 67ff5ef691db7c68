"""Newtonian (leading post-Newtonian order) chirp injections.

The paper injects IMRPhenomPv2 waveforms (Sec. IV.B); that approximant is a
third-party model, so the stand-in is the quadrupole-order inspiral chirp:
frequency f(tau) = (1/pi) (5 / (256 tau))^(3/8) Mc^(-5/8) and amplitude
proportional to tau^(-1/4), with tau = t_c - t and Mc = G M_chirp / c^3 in
seconds.  Each detector sees the chirp with its own random phase and relative
amplitude; the pair is then rescaled to a target network SNR (the quadrature
sum of the per-detector SNRs, as the paper defines it in its introduction).
"""
import numpy as np

from .noise import analytic_psd

T_SUN = 4.925491e-6  # G M_sun / c^3 in seconds


def _tau_of_f(f, mc_s):
    return (5.0 / 256.0) * mc_s ** (-5.0 / 3.0) * (np.pi * f) ** (-8.0 / 3.0)


def newtonian_chirp(mchirp_msun, fs=2048.0, f_low=20.0, f_high=1000.0, taper_s=0.1):
    """Return (h, n_after): chirp samples and the gap from its last sample to t_c.

    The chirp runs from f_low to min(f_ISCO, f_high); f_ISCO uses the equal-mass
    total mass M = Mc 4^(3/5).  Sample i sits at t = t_c - tau_i with
    tau_i = tau(f_low) - i / fs, and the series stops where f reaches f_end,
    n_after samples before t_c.  h is tapered with half-Hann ramps (taper_s at
    the start, four cycles of the final frequency at the end); its overall scale
    is arbitrary because injections are rescaled to a target SNR.
    """
    mc_s = mchirp_msun * T_SUN
    m_tot_s = mc_s * 4.0 ** 0.6
    f_isco = 1.0 / (6.0 ** 1.5 * np.pi * m_tot_s)
    f_end = min(f_isco, f_high)
    tau0 = _tau_of_f(f_low, mc_s)
    tau1 = _tau_of_f(f_end, mc_s)
    n = int(np.floor((tau0 - tau1) * fs))
    tau = tau0 - np.arange(n) / fs
    phase = -2.0 * (tau / (5.0 * mc_s)) ** 0.625
    h = tau ** -0.25 * np.cos(phase)
    w = np.ones(n)
    n_a = min(int(taper_s * fs), n // 2)
    if n_a > 0:
        w[:n_a] = 0.5 - 0.5 * np.cos(np.pi * np.arange(n_a) / n_a)
    n_b = min(int(4.0 / f_end * fs), n // 2)
    if n_b > 0:
        w[n - n_b:] = 0.5 + 0.5 * np.cos(np.pi * (np.arange(n_b) + 1) / n_b)
    # samples of h are at times t_c - tau; the last one sits tau1 before t_c
    return h * w, int(round(tau1 * fs))


def _snr2(h, fs, f_lo=32.0, f_hi=1024.0, n_fft=65536):
    """rho^2 = 4 int |h~(f)|^2 / S(f) df over [f_lo, f_hi], on a zero-padded
    grid fine enough (32 s) that the band edge at f_lo is resolved."""
    n = max(len(h), n_fft)
    spec = np.fft.rfft(h, n=n) / fs
    f = np.arange(len(spec)) * fs / n
    s = analytic_psd(f)
    band = (f >= f_lo) & (f <= f_hi) & (s > 0)
    return 4.0 * np.sum(np.abs(spec[band]) ** 2 / s[band]) * (fs / n)


def inject_chirps(x, fs=2048.0, first_tc=None, spacing_s=60.0, seed=0,
                  mc_range=(10.0, 60.0), snr_range=(4.0, 20.0), amp_range=(0.1, 1.0)):
    """Add chirps to x [2, n] (float64, physical strain) in place; return a list
    of dicts with t_c sample index, chirp mass and target/actual network SNR."""
    rng = np.random.default_rng(seed)
    n = x.shape[1]
    tc = int(first_tc if first_tc is not None else spacing_s * fs)
    out = []
    while tc < n:
        mc = rng.uniform(*mc_range)
        snr = rng.uniform(*snr_range)
        base, n_after = newtonian_chirp(mc, fs)
        hs = []
        for _ in range(x.shape[0]):
            ph = rng.uniform(0.0, 2.0 * np.pi)
            amp = rng.uniform(*amp_range)
            # a phase rotation of the carrier: real part of amp * e^{i ph} * analytic chirp
            analytic = np.fft.ifft(np.fft.fft(base) * _hilbert_mask(len(base)))
            hs.append(amp * np.real(np.exp(1j * ph) * analytic))
        rho2 = sum(_snr2(h, fs) for h in hs)
        g = snr / np.sqrt(rho2)
        end = tc - n_after
        start = end - len(base)
        lo = max(start, 0)
        hi = min(end, n)
        if hi > lo:
            for c in range(x.shape[0]):
                x[c, lo:hi] += g * hs[c][lo - start:hi - start]
        out.append({"tc": tc, "mchirp": mc, "snr": snr})
        tc += int(spacing_s * fs)
    return out


def _hilbert_mask(n):
    m = np.zeros(n)
    m[0] = 1.0
    if n % 2 == 0:
        m[n // 2] = 1.0
        m[1:n // 2] = 2.0
    else:
        m[1:(n + 1) // 2] = 2.0
    return m
