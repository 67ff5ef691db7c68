"""GPU: af_whiten_noalloc (static scratch, no allocation) against af_whiten
(caller's workspace) through the C ABI: the same output bit for bit, on two
calls in a row, the second smaller; requests beyond the scratch are rejected."""
import ctypes

import numpy as np
import pytest

from synth.noise import coloured_noise
from tests.gpu_util import banner, dev, need_gpu

pytestmark = pytest.mark.gpu
FS, PRESCALE = 2048.0, 1e21


def noalloc(P, x, psd, n_psd, hop, out_start, n_out, y):
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return P.lib().af_whiten_noalloc(ctypes.c_void_p(x.data_ptr()), 0, x.shape[0], x.shape[1], x.stride(0), FS,
                                     PRESCALE, ctypes.c_void_p(psd.data_ptr()), 4096, n_psd, hop, 1.0, 32.0,
                                     out_start, n_out, ctypes.c_void_p(y.data_ptr()), y.stride(0), s)


def test_noalloc_equals_workspace_form():
    P = need_gpu()
    import torch
    fs = int(FS)
    M = fs // 2
    cases = [(96, 3, 8 * fs, 2, 31), (70, 1, 0, 1, 32)]   # seconds, PSDs, hop, channels, seed: second smaller
    for secs, n_psd, hop, n_ch, seed in cases:
        banner(f"whiten noalloc {secs} s, {n_psd} PSDs, {n_ch} ch")
        x = dev(coloured_noise(fs * secs, seed=seed)[:n_ch])
        psd = P.psd_estimate(x, FS, PRESCALE, psd_len=64 * fs, psd_hop=hop, n_psd=n_psd)
        out_start = 64 * fs + M
        n_out = x.shape[1] - out_start - M
        ref = P.whiten(x, psd, FS, PRESCALE, hop, out_start=out_start, n_out=n_out)
        y = torch.full_like(ref, float("nan"))
        P.check(noalloc(P, x, psd, n_psd, hop, out_start, n_out, y))
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
    # 513 PSDs of two detectors need more than the 16 MiB scratch
    x = dev(coloured_noise(fs * 80, seed=33))
    big = torch.ones((513, 2, 2049), dtype=torch.float64, device="cuda")
    y = torch.empty((2, 513 * 16), dtype=torch.float32, device="cuda")
    rc = noalloc(P, x, big, 513, 16, M, 513 * 16, y)
    assert rc == -1 and b"static scratch" in P.lib().af_last_error()
