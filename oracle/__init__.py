"""FP64 CPU oracle for the whitening + 1D-ResNet scoring path (test infrastructure).

This package is a plain, slow, obviously correct NumPy implementation of what
the GPU library computes, written from the paper's description of the method
(Welch PSD, inverse-ASD whitening filter with 0.5 s settle-in per edge,
windowed residual-CNN scoring (also in the GroupNorm form), 1 s top-hat integration, clustering into
candidate events and their false alarm rates, projection of injections onto
the detectors and their network SNR).  It exists only to
check the GPU path: it is imported by the test-suite, by the smoke check and by
the benchmark's CPU-baseline leg, never by the library itself.  It shares no
code with the HIP path; the only common module is `synth`, which generates the
seeded inputs and holds none of the method's arithmetic.

Parity status: every function here is pinned by tests/test_oracle_*.py against
closed forms, brute-force sums, library routines or invariants; see each
module's header.
"""
from .welch import hann_periodic, welch_psd, welch_psd_rolling, periodogram_dft
from .whiten import whitening_fir, whiten, whiten_piecewise, whiten_at
from .net import fold_bn, conv1d, net_forward, net_forward_quant
from .net_gn import group_norm, net_forward_gn
from .post import integrate, kendall_tau_b, unfold_windows
from .quant import bf16_round, e4m3_round
from .events import cluster, false_alarm_rate
from .inject import antenna, project, network_snr

__all__ = [
    "hann_periodic", "welch_psd", "welch_psd_rolling", "periodogram_dft",
    "whitening_fir", "whiten", "whiten_piecewise", "whiten_at",
    "fold_bn", "conv1d", "net_forward", "net_forward_quant", "group_norm", "net_forward_gn",
    "integrate", "kendall_tau_b", "unfold_windows", "bf16_round", "e4m3_round",
    "cluster", "false_alarm_rate", "antenna", "project", "network_snr",
]
