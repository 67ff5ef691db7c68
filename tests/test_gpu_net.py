"""GPU parity: score_windows (implicit-GEMM MFMA ResNet-1D) against the FP64
oracle and against its quantisation-emulating variant."""
import numpy as np
import pytest
import torch

import oracle
from synth import RESNET_ARCH, TINY_ARCH, make_params
from synth.params import NetArch
from tests.gpu_util import banner, dev, need_gpu

pytestmark = pytest.mark.gpu

# logit tolerances against the FP64 oracle, per precision
TOL = {"f32": 1e-3, "bf16": 3e-2, "bf16f": 3e-2, "fp8": 1e-1}
# tiny net against the quantisation-emulating oracle
EMU_TOL = {"bf16": 2e-5, "bf16f": 2e-5, "fp8": 5e-4}


def series(n, seed, n_ch=2):
    """A unit-variance float32 series standing in for whitened strain."""
    return np.random.default_rng(seed).standard_normal((n_ch, n)).astype(np.float32)


# calibration windows of FP8 nets: 16 windows of unit-variance noise (the
# statistics of whitened strain), not the windows under test
CALIB_STRIDE = 1000


def calib_series(window=3072, n=16):
    return series(window + CALIB_STRIDE * (n - 1), seed=99)


def calib_windows(window=3072, n=16):
    return oracle.unfold_windows(calib_series(window, n).astype(np.float64), window, CALIB_STRIDE)[:n]


def oracle_logits(params, arch, y, stride, nw, shifts=None, wrap=0, precision=None, calib=False):
    w = oracle.unfold_windows(y.astype(np.float64), arch.window, stride, shifts, wrap)[:nw]
    if precision in (None, "f32"):
        return oracle.net_forward(params, arch, w)
    return oracle.net_forward_quant(params, arch, w, precision,
                                    calib=calib_windows(arch.window) if calib else None)


def make_net(P, arch, params, prec):
    """A scoring net; FP8 nets are bias-corrected on the calibration windows."""
    net = P.Net(arch, params, prec)
    if prec == "fp8":
        net.calibrate(dev(calib_series(arch.window)), CALIB_STRIDE)
    return net


@pytest.mark.parametrize("arch,prec", [(TINY_ARCH, "f32"), (TINY_ARCH, "bf16"), (TINY_ARCH, "bf16f"),
                                       (TINY_ARCH, "fp8"), (RESNET_ARCH, "f32"), (RESNET_ARCH, "bf16"),
                                       (RESNET_ARCH, "bf16f"), (RESNET_ARCH, "fp8")],
                         ids=["tiny-f32", "tiny-bf16", "tiny-bf16f", "tiny-fp8", "resnet-f32", "resnet-bf16",
                              "resnet-bf16f", "resnet-fp8"])
def test_logits_vs_fp64(arch, prec):
    P = need_gpu()
    banner(f"score {arch.name} {prec}")
    params = make_params(arch, seed=0)
    nw = 12 if arch is RESNET_ARCH else 24
    stride = 128
    y = series(arch.window + stride * (nw - 1) + 77, seed=1)
    net = make_net(P, arch, params, prec)
    got = net.score_windows(dev(y), stride, nw, batch=5).cpu().numpy()
    ref = oracle_logits(params, arch, y, stride, nw)
    err = np.abs(got - ref).max()
    print(f"max|dlogit| {prec} {arch.name}: {err:.3e}")
    assert err < TOL[prec]
    if prec != "f32":
        emu = oracle_logits(params, arch, y, stride, nw, precision=prec, calib=prec == "fp8")
        e2 = np.abs(got - emu).max()
        print(f"max|dlogit| vs emulation: {e2:.3e}")
        # The emulation takes every rounding decision at the same points as the
        # kernel, but its sums are FP64 while the MFMA sums in FP32; rare
        # decision flips then propagate layer to layer.  For the 5-conv tiny net
        # that stays at rounding level; for the 37-conv ResNet it grows to the
        # size of the precision's own error, so there the FP64 bound applies.
        assert e2 < (EMU_TOL[prec] if arch is TINY_ARCH else TOL[prec])


def test_fp32_logits_tight_tiny():
    P = need_gpu()
    params = make_params(TINY_ARCH, seed=2)
    y = series(3072 + 64 * 40, seed=3)
    got = P.Net(TINY_ARCH, params, "f32").score_windows(dev(y), 64).cpu().numpy()
    ref = oracle_logits(params, TINY_ARCH, y, 64, len(got))
    assert len(got) == 41
    np.testing.assert_allclose(got, ref, atol=2e-5, rtol=1e-5)


def test_shifts_and_wrap():
    # channel 1 shifted circularly (a timeslide): same as the oracle on the remapped windows
    P = need_gpu()
    banner("score shifts+wrap")
    params = make_params(TINY_ARCH, seed=4)
    n = 3072 * 4
    y = series(n, seed=5)
    shifts = [0, 2048 * 3]
    got = P.Net(TINY_ARCH, params, "f32").score_windows(dev(y), 2048, 5, shifts=shifts, wrap=n).cpu().numpy()
    ref = oracle_logits(params, TINY_ARCH, y, 2048, 5, np.array(shifts), n)
    np.testing.assert_allclose(got, ref, atol=2e-5, rtol=1e-5)
    # the strided, pooled ResNet stem reads the same circular windows
    rp = make_params(RESNET_ARCH, seed=29)
    got = P.Net(RESNET_ARCH, rp, "f32").score_windows(dev(y), 2048, 5, shifts=shifts, wrap=n).cpu().numpy()
    ref = oracle_logits(rp, RESNET_ARCH, y, 2048, 5, np.array(shifts), n)
    assert np.abs(got - ref).max() < TOL["f32"]
    with pytest.raises(P.AframeError, match="EINVAL"):   # a wrap shorter than a window
        P.Net(TINY_ARCH, params, "f32").score_windows(dev(y), 2048, 1, shifts=shifts, wrap=3000)


def test_edge_cases():
    P = need_gpu()
    params = make_params(TINY_ARCH, seed=6)
    net = P.Net(TINY_ARCH, params, "f32")
    y = dev(series(3072, seed=7))
    assert net.score_windows(y, 128, 0).numel() == 0
    one = net.score_windows(y, 128, 1).cpu().numpy()
    ref = oracle_logits(params, TINY_ARCH, y.cpu().numpy(), 128, 1)
    np.testing.assert_allclose(one, ref, atol=2e-5)
    with pytest.raises(P.AframeError, match="EINVAL"):
        net.score_windows(y, 128, 2)           # second window runs past the end


def test_deterministic_across_batches():
    # a window's logit does not depend on which batch it runs in
    P = need_gpu()
    params = make_params(RESNET_ARCH, seed=8)
    y = dev(series(3072 + 128 * 20, seed=9))
    net = P.Net(RESNET_ARCH, params, "bf16")
    a = net.score_windows(y, 128, 21, batch=21).cpu().numpy()
    b = net.score_windows(y, 128, 21, batch=4).cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_fp8_calibration():
    # bias correction on the GPU (FP32 twin for the input means and the FC
    # shift) against the oracle's (FP64 net), on a shallow net the emulation
    # pins tightly; repeated calibration gives the same logits bit for bit;
    # only FP8 nets calibrate
    P = need_gpu()
    banner("fp8 calibration")
    arch = SHALLOW[1]
    params = make_params(arch, seed=25)
    y = series(3072 + 128 * 7, seed=26)
    net = P.Net(arch, params, "fp8")
    plain = net.score_windows(dev(y), 128).cpu().numpy()
    net.calibrate(dev(calib_series()), CALIB_STRIDE)
    got = net.score_windows(dev(y), 128).cpu().numpy()
    emu = oracle_logits(params, arch, y, 128, len(got), precision="fp8", calib=True)
    emu_plain = oracle_logits(params, arch, y, 128, len(got), precision="fp8")
    print(f"calibrated vs emulation {np.abs(got - emu).max():.2e}; the correction moves the logits by "
          f"{np.abs(emu - emu_plain).max():.2e} (GPU {np.abs(got - plain).max():.2e})")
    assert np.abs(got - emu).max() < 2e-3
    net.calibrate(dev(calib_series()), CALIB_STRIDE)
    np.testing.assert_array_equal(net.score_windows(dev(y), 128).cpu().numpy(), got)
    for prec in ("f32", "bf16", "bf16f"):
        with pytest.raises(P.AframeError, match="EINVAL"):
            P.Net(arch, params, prec).calibrate(dev(calib_series()), CALIB_STRIDE)


def test_fused_tiny_matches_layer_path():
    # the persistent whole-network kernel and the layer-by-layer kernels agree
    P = need_gpu()
    banner("fused tiny bf16 vs layer path")
    params = make_params(TINY_ARCH, seed=21)
    y = dev(series(3072 + 128 * 40, seed=22))
    net = P.Net(TINY_ARCH, params, "bf16")
    assert net.fused
    a = net.score_windows(y, 128).cpu().numpy()
    net.fused = False
    b = net.score_windows(y, 128, batch=16).cpu().numpy()
    net.fused = True
    assert np.abs(a - b).max() < 2e-5
    ref = oracle_logits(params, TINY_ARCH, y.cpu().numpy(), 128, len(a), precision="bf16")
    assert np.abs(a - ref).max() < EMU_TOL["bf16"]


def test_fused_step_candidates_same_logits():
    # every rows-per-step candidate of the whole-network kernel gives the same
    # logits bit for bit (windows of every length class: one, a few, ragged)
    P = need_gpu()
    banner("fused tiny step candidates")
    params = make_params(TINY_ARCH, seed=30)
    y = dev(series(3072 + 128 * 70 + 5, seed=31))
    net = P.Net(TINY_ARCH, params, "bf16")
    rows, n_cand, chosen = net.fused_tile()
    ref = net.score_windows(y, 128).cpu().numpy()
    for c in range(n_cand):
        net.set_fused_tile(c)
        assert net.fused_tile()[0] in (32, 48, 64)
        np.testing.assert_array_equal(net.score_windows(y, 128).cpu().numpy(), ref)
        np.testing.assert_array_equal(net.score_windows(y, 128, 1).cpu().numpy(), ref[:1])
    net.set_fused_tile(chosen)
    changed = net.autotune(batch=256)
    print(f"fused rows per step: {net.fused_tile()}, autotune changed {changed}")
    np.testing.assert_array_equal(net.score_windows(y, 128).cpu().numpy(), ref)
    with pytest.raises(P.AframeError, match="EINVAL"):
        net.set_fused_tile(n_cand)


def test_fused_unavailable_for_fp32():
    P = need_gpu()
    net = P.Net(TINY_ARCH, make_params(TINY_ARCH, seed=1), "f32")
    assert not net.fused
    with pytest.raises(P.AframeError, match="EINVAL"):
        net.fused = True


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16f"])
def test_autotune_keeps_logits(prec):
    # switching tile shapes leaves every window's arithmetic unchanged
    P = need_gpu()
    banner(f"autotune resnet {prec}")
    params = make_params(RESNET_ARCH, seed=23)
    y = dev(series(3072 + 128 * 15, seed=24))
    net = P.Net(RESNET_ARCH, params, prec)
    before = net.score_windows(y, 128).cpu().numpy()
    changed = net.autotune(batch=64)
    tiles = net.tiles()
    assert len(tiles) == 35 and all(0 <= t[3] < t[2] for t in tiles if t[2] > 0)
    after = net.score_windows(y, 128).cpu().numpy()
    print(f"autotune changed {changed} layers")
    np.testing.assert_allclose(after, before, atol=1e-5 if prec == "f32" else 2e-3)


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16f", "fp8"])
def test_every_tile_candidate_same_logits(prec):
    # every tile shape the autotuner may choose, layer by layer, gives the
    # logits of the default shape bit for bit (the k summation order does not
    # depend on the tiling)
    P = need_gpu()
    banner(f"tile candidates resnet {prec}")
    params = make_params(RESNET_ARCH, seed=27)
    y = dev(series(3072 + 128 * 5, seed=28))
    net = P.Net(RESNET_ARCH, params, prec)
    ref = net.score_windows(y, 128, batch=3).cpu().numpy()
    tried = 0
    for layer, (_, _, n_cand, chosen) in enumerate(net.tiles(), start=1):
        for c in range(n_cand):
            if c == chosen:
                continue
            net.set_tile(layer, c)
            got = net.score_windows(y, 128, batch=3).cpu().numpy()
            assert np.array_equal(got, ref), f"layer {layer} candidate {c}: max|d| {np.abs(got - ref).max():.3e}"
            tried += 1
        net.set_tile(layer, chosen)
    print(f"{prec}: {tried} alternative tiles, all identical")
    with pytest.raises(P.AframeError, match="EINVAL"):
        net.set_tile(1, net.tiles()[0][2])
    with pytest.raises(P.AframeError, match="EINVAL"):
        net.set_tile(0, 0)


SHALLOW = [NetArch("shallow32", 2, 32, 7, 2, True, (32,), (1,)),
           NetArch("shallow64", 2, 32, 7, 2, True, (32, 64), (1, 1)),
           NetArch("shallow128", 2, 32, 7, 2, True, (32, 64, 128), (1, 1, 1))]


# FP8 gaps grow faster with depth than BF16's (measured 1.5e-5, 3.0e-4 and
# 1.6e-3 for the three nets): where FP32 and FP64 sums round a window's
# largest activation to different BF16 neighbours, that window's activation
# scale for the next conv moves, and with it the E4M3 rounding of many operands.
@pytest.mark.parametrize("prec,tol", [("bf16", 2e-4), ("bf16f", 2e-4), ("fp8", 2e-3)])
@pytest.mark.parametrize("arch", SHALLOW, ids=lambda a: a.name)
def test_shallow_resnets_vs_emulation(arch, prec, tol):
    # every low-precision layer kind (stride-1 k7 with the tap-shift operand
    # reuse, stride-2 k7, 1x1 projection, 32/64/128 wide) against the
    # quantisation-emulating oracle on nets shallow enough for it to pin tightly
    P = need_gpu()
    banner(f"shallow {arch.name} {prec}")
    params = make_params(arch, seed=25)
    y = series(3072 + 128 * 7, seed=26)
    got = P.Net(arch, params, prec).score_windows(dev(y), 128).cpu().numpy()
    emu = oracle_logits(params, arch, y, 128, len(got), precision=prec)
    print(f"{arch.name} {prec}: max|d| vs emulation {np.abs(got - emu).max():.2e}")
    assert np.abs(got - emu).max() < tol
