"""GPU parity of whitening at the 24 h size (the benchmark's whitening
workload: 24 independently coloured hours of two-detector noise, rolling 64 s
PSD every 8 s, 1 s FIR, 32 Hz high-pass), checked on sampled PSD hops and on
spans of the whitened series that the FP64 oracle recomputes sample by sample:
the first and last outputs, block and hop boundaries, and the junctions of the
coloured hours."""
import numpy as np
import pytest
import torch

import oracle
from synth.noise import coloured_noise
from synth.workloads import PSD_LEN
from tests.gpu_util import banner, need_gpu, rel_l2

pytestmark = pytest.mark.gpu
FS = 2048.0
HOP, M = 16384, 1024


@pytest.fixture(scope="module")
def day_run():
    P = need_gpu()
    from paper_2403_18661_amd.pipeline import OfflinePath, PathConfig
    from synth import TINY_ARCH, make_params
    banner("whitening, 24 h")
    x = np.concatenate([coloured_noise(3600 * int(FS), seed=7000 + h) for h in range(24)], axis=1)
    net = P.Net(TINY_ARCH, make_params(TINY_ARCH, seed=0), "bf16")   # only sizes the path's buffers
    path = OfflinePath(net, x.shape[1], PathConfig(psd_len=PSD_LEN), batch=1)
    xd = torch.from_numpy(x).cuda()
    path.psd_stage(xd)
    path.response_stage()
    path.apply_stage(xd)
    torch.cuda.synchronize()
    return {"x": x, "path": path}


def test_day_counts(day_run):
    path, x = day_run["path"], day_run["x"]
    assert path.n_out == x.shape[1] - PSD_LEN - 2 * M
    assert path.n_psd == -(-path.n_out // HOP) == 10792


@pytest.mark.parametrize("j", [0, 5396, 10791])
def test_day_sampled_psd(day_run, j):
    x = day_run["x"]
    ref = oracle.welch_psd(x[:, j * HOP: j * HOP + PSD_LEN] * 1e21, FS)
    np.testing.assert_allclose(day_run["path"].psd[j].cpu().numpy(), ref, rtol=1e-10)


def test_day_sampled_spans(day_run):
    x, path = day_run["x"], day_run["path"]
    n_out = path.n_out
    n0 = PSD_LEN + M
    hour = 3600 * int(FS)
    starts = [0, 6146 - 32, HOP - 32, 5396 * HOP - 32, 12 * hour - n0 - 32, n_out - 64]
    y = path.y
    for i0 in starts:
        span = np.arange(i0, i0 + 64)
        got = y[:, i0:i0 + 64].cpu().numpy()
        for c in range(2):
            ref = np.empty(64)
            for j in np.unique(span // HOP):
                sel = span // HOP == j
                psd = oracle.welch_psd(x[:, j * HOP: j * HOP + PSD_LEN], FS)
                taps = oracle.whitening_fir(psd, FS)
                ref[sel] = oracle.whiten_at(x[c], taps[c], n0 + span[sel], FS)
            err = rel_l2(got[c], ref)
            print(f"span at {i0}, channel {c}: relative L2 {err:.2e}")
            assert err < 1e-5
