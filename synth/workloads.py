"""Seeded workloads (input recipes only).

* tiny (plain path): 2 detectors x 16 s of noise with the analytic PSD, seed 0.
* hour (plain path, full size): 1 h of analysed output at 16 Hz (57,600 windows
  of 3072 samples), preceded by the 64 s PSD background and 0.5 s filter
  context and followed by 0.5 s of filter context; Newtonian chirps every 60 s
  with chirp mass U(10, 60) Msun and network SNR U(4, 20).
"""
import numpy as np

from .chirps import inject_chirps
from .noise import coloured_noise

FS = 2048
WINDOW = 3072
STRIDE = 128
PSD_LEN = 64 * FS
FIR_HALF = FS // 2


def hour_length(n_windows=57600, window=WINDOW, stride=STRIDE):
    """Raw samples per detector for the full-size workload."""
    n_out = (n_windows - 1) * stride + window
    return PSD_LEN + FIR_HALF + n_out + FIR_HALF


def tiny_strain(seed=0):
    return coloured_noise(16 * FS, seed=seed)


def hour_strain(seed=0, n_windows=57600, chirps=True):
    n = hour_length(n_windows)
    x = coloured_noise(n, seed=seed)
    inj = inject_chirps(x, seed=seed + 1000) if chirps else []
    return x, inj
