"""Writes tests/golden/hour_integrated_fp64.npy: the FP64 oracle's integrated
statistic of the whole hour workload (57,600 windows at 16 Hz, 57,585
integrated values), the reference of the rank-agreement test of every
precision on that workload.  It calls only oracle/ (and synth/ for the seeded
inputs): rolling 64 s Welch PSD every 8 s, piecewise FIR whitening, the FP64
ResNet forward, 16-window integration.

    python -m tests.golden.make_hour_fp64        (about half an hour on 8 cores)
"""
import os
import sys

import numpy as np

import oracle
from synth import RESNET_ARCH, make_params
from synth.workloads import PSD_LEN, hour_strain

FS = 2048.0
HOP, M, WIN, STRIDE, N_WIN, WIDTH = 16384, 1024, 3072, 128, 57600, 16
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hour_integrated_fp64.npy")


def main(chunk=512):
    x, _ = hour_strain(seed=0)
    params = make_params(RESNET_ARCH, seed=0)
    n_out = (N_WIN - 1) * STRIDE + WIN
    n_psd = -(-n_out // HOP)
    psds = oracle.welch_psd_rolling(x, FS, PSD_LEN, HOP, n_psd)
    y = oracle.whiten_piecewise(x, psds, FS, PSD_LEN + M, n_out, HOP)
    logits = np.empty(N_WIN)
    for w0 in range(0, N_WIN, chunk):
        n = min(chunk, N_WIN - w0)
        span = y[:, w0 * STRIDE: (w0 + n - 1) * STRIDE + WIN]
        logits[w0:w0 + n] = oracle.net_forward(params, RESNET_ARCH, oracle.unfold_windows(span, WIN, STRIDE))
        print(f"{w0 + n} / {N_WIN} windows", file=sys.stderr, flush=True)
    np.save(OUT, oracle.integrate(logits, WIDTH))


if __name__ == "__main__":
    main()
