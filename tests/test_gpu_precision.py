"""GPU: the precision workload — the tiny plain path (16 s, 217 windows) with
the convs in BF16 and FP8 — errors per stage against the FP64 oracle and the
rank agreement (Kendall tau-b) of the integrated statistic."""
import numpy as np
import pytest
import torch

import oracle
from synth import TINY_ARCH, make_params
from synth.workloads import tiny_strain
from tests.gpu_util import banner, need_gpu, rel_l2

pytestmark = pytest.mark.gpu
FS = 2048.0
TOL = {"f32": 1e-3, "bf16": 3e-2, "bf16f": 3e-2, "fp8": 1e-1}


@pytest.fixture(scope="module")
def reference():
    x = tiny_strain(seed=0)
    params = make_params(TINY_ARCH, seed=0)
    y = oracle.whiten(x, oracle.welch_psd(x, FS), FS)
    logits = oracle.net_forward(params, TINY_ARCH, oracle.unfold_windows(y, 3072, 128))
    return {"x": x, "params": params, "y": y, "logits": logits, "integ": oracle.integrate(logits, 16)}


FP8_TAU = pytest.param("fp8", marks=pytest.mark.xfail(strict=False, reason=(
    "FP8 rank agreement on 16 s of noise: the integrated statistic of the random-init net varies by "
    "~0.011 across windows; rounding the activations alone to E4M3 (weights exact) already gives tau "
    "0.984 in emulation, and bias correction removes only the weight rounding's systematic shift "
    "(emulated tau 0.982 with it)")))


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16f", FP8_TAU])
def test_precision_workload(reference, prec):
    P = need_gpu()
    banner(f"precision workload {prec}")
    xd = torch.from_numpy(reference["x"]).cuda()
    y = P.whiten(xd, P.psd_estimate(xd, FS, 1e21), FS, 1e21)
    net = P.Net(TINY_ARCH, reference["params"], prec)
    if prec == "fp8":
        c = np.random.default_rng(99).standard_normal((2, 3072 + 1000 * 15)).astype(np.float32)
        net.calibrate(torch.from_numpy(c).cuda(), 1000)
    logits = net.score_windows(y, 128)
    integ = P.integrate(logits, 16).cpu().numpy()
    yg, lg = y.cpu().numpy(), logits.cpu().numpy()
    werr = max(rel_l2(yg[c], reference["y"][c]) for c in range(2))
    lerr = np.abs(lg - reference["logits"]).max()
    tau = oracle.kendall_tau_b(integ, reference["integ"])
    print(f"{prec}: whitened rel L2 {werr:.2e}, max|dlogit| {lerr:.2e}, tau {tau:.4f}, "
          f"integrated spread {reference['integ'].std():.4f}")
    assert werr < 1e-5
    assert lerr < TOL[prec]
    assert tau >= 0.99
