"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package holds input generation only: coloured Gaussian noise, Newtonian
chirp injections, lognormal segment layouts and randomly initialised network
parameters.  It contains none of the detection method's arithmetic (no PSD
estimation, whitening, convolution or integration), so it can feed both the
FP64 oracle and the HIP library without coupling them.  The one spectral sum it
computes, the SNR that sets each injected chirp's amplitude (chirps._snr2), is
part of the input recipe: neither the oracle nor the library calls it.
"""
from .noise import analytic_psd, coloured_noise
from .chirps import newtonian_chirp, inject_chirps
from .segments import lognormal_segments
from .params import NetArch, TINY_ARCH, RESNET_ARCH, GN_ARCH, GN_NARROW_ARCH, TINY_GN_ARCH, make_params

__all__ = [
    "analytic_psd", "coloured_noise", "newtonian_chirp", "inject_chirps",
    "lognormal_segments", "NetArch", "TINY_ARCH", "RESNET_ARCH", "GN_ARCH", "GN_NARROW_ARCH", "TINY_GN_ARCH", "make_params",
]
