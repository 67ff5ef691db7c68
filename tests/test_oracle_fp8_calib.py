"""Pins of the E4M3 bias correction in the oracle (oracle.net: conv_input_means,
fp8_bias_shift, net_forward_quant with calibration windows)."""
from collections import OrderedDict

import numpy as np
import pytest
import torch

import oracle
from oracle.net import conv_input_means, fp8_bias_shift
from synth import RESNET_ARCH, TINY_ARCH, make_params
from synth.params import NetArch
from tests.test_oracle_net import torch_model

TWO_CH = NetArch("pin2ch", in_ch=2, stem_ch=2, kernel=1, stem_stride=1, stem_pool=False,
                 widths=(2,), blocks=(1,), window=4)


def two_channel_params():
    """Identity BatchNorms (folded scale 1, bias 0), identity stem, and conv
    weights with one entry off the E4M3 grid per first row."""
    par = OrderedDict()

    def conv(name, w):
        par[name + ".w"] = np.asarray(w, dtype=np.float64)[:, :, None]

    def bn(name):
        par[name + ".gamma"] = np.full(2, np.sqrt(1.0 + 1e-5))
        par[name + ".beta"] = np.zeros(2)
        par[name + ".mean"] = np.zeros(2)
        par[name + ".var"] = np.ones(2)

    conv("stem.conv", [[1.0, 0.0], [0.0, 1.0]]); bn("stem.bn")
    conv("s0.b0.conv1", [[448.0, 1.0625], [1.0, 1.0]]); bn("s0.b0.bn1")
    conv("s0.b0.conv2", [[2.0, 0.2], [0.0, 1.0]]); bn("s0.b0.bn2")
    par["fc.w"] = np.ones((1, 2))
    par["fc.b"] = np.zeros(1)
    return par


def test_hand_worked_shifts():
    # Input constant 1 and 2 on the two channels: the stem passes it, so conv1's
    # input means are (1, 2).  conv1 row 0 has scale 448/448 = 1 and 1.0625
    # lies halfway between the E4M3 values 1 and 1.125: it rounds to 1 (even),
    # a weight error of -1/16 on channel 1, so row 0 moves by -1/16 * 2 = -1/8;
    # row 1 (1, 1) scales to (448, 448), exact.  conv2's input is conv1's FP64
    # output (448 + 2.125, 3); its row 0 has scale 2/448, 0.2 scales to 44.8,
    # which rounds to 44 (grid step 4 on [32, 64)): the weight becomes
    # 44 * 2/448 = 11/56, an error of 11/56 - 1/5 = -1/280, so row 0 moves by
    # -3/280; row 1 (0, 1) is exact.
    par = two_channel_params()
    x = np.array([[[1.0] * 4, [2.0] * 4]])
    mu = conv_input_means(par, TWO_CH, x)
    np.testing.assert_array_equal(mu["s0.b0.conv1"], [1.0, 2.0])
    np.testing.assert_array_equal(mu["s0.b0.conv2"], [450.125, 3.0])
    shift = fp8_bias_shift(par, TWO_CH, x)
    np.testing.assert_allclose(shift["s0.b0.conv1"], [-0.125, 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(shift["s0.b0.conv2"], [-3.0 / 280.0, 0.0], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("arch", [TINY_ARCH, RESNET_ARCH], ids=lambda a: a.name)
def test_input_means_match_torch_forward_hooks(arch):
    # the conv inputs, read out of an independently assembled torch.nn model
    params = make_params(arch, seed=5)
    x = np.random.default_rng(6).standard_normal((3, 2, 3072))
    run = torch_model(arch, params)
    model = run.model
    seen = {}

    def hook(name):
        return lambda mod, inp, out: seen.__setitem__(name, inp[0].mean(dim=(0, 2)).numpy())

    for blk, (pre, _, _, _, p) in zip(model["blocks"], arch.block_list()):
        blk.conv1.register_forward_hook(hook(pre + ".conv1"))
        blk.conv2.register_forward_hook(hook(pre + ".conv2"))
        if p:
            blk.proj[0].register_forward_hook(hook(pre + ".proj"))
    run(x)
    mu = conv_input_means(params, arch, x)
    assert set(mu) == set(seen)
    for k in mu:
        np.testing.assert_allclose(mu[k], seen[k], rtol=1e-10, atol=1e-12)


def test_fc_shift_centres_the_calibration_logits():
    # evaluated on its own calibration windows, the corrected network's mean
    # logit equals the FP64 network's mean logit (up to the FP32 rounding of
    # the shifted FC bias, |shift| 2^-24 < 1e-9)
    params = make_params(TINY_ARCH, seed=0)
    x = np.random.default_rng(7).standard_normal((4, 2, 3072)).astype(np.float32).astype(np.float64)
    got = oracle.net_forward_quant(params, TINY_ARCH, x, "fp8", calib=x)
    ref = oracle.net_forward(params, TINY_ARCH, x)
    assert abs(got.mean() - ref.mean()) < 1e-9
    assert abs(oracle.net_forward_quant(params, TINY_ARCH, x, "fp8").mean() - ref.mean()) > 1e-3


def test_weights_on_the_grid_need_no_shift():
    params = make_params(TINY_ARCH, seed=1)
    L = oracle.net.folded_layers(params, TINY_ARCH)
    for pre, _, _, _, _ in TINY_ARCH.block_list():
        for c in (".conv1", ".conv2"):
            w = L[pre + c][0]
            g = oracle.net.fp8_weights(w)
            # put the folded weights on their own E4M3 grid: undo the fold's scale
            s = params[pre + (".bn1" if c == ".conv1" else ".bn2") + ".gamma"] / np.sqrt(
                params[pre + (".bn1" if c == ".conv1" else ".bn2") + ".var"] + 1e-5)
            params[pre + c + ".w"] = g / s[:, None, None]
    x = np.random.default_rng(8).standard_normal((2, 2, 3072))
    for name, v in fp8_bias_shift(params, TINY_ARCH, x).items():
        assert np.abs(v).max() < 1e-12 * max(1.0, np.abs(conv_input_means(params, TINY_ARCH, x)[name]).max())


def test_correction_brings_the_resnet_within_the_fp8_bar():
    # emulated E4M3 ResNet of the hour workload: the weight rounding shifts the
    # logits by ~0.07 on every window; the correction (calibrated on other
    # noise) removes the shift and leaves the logits within the 1e-1 bar
    params = make_params(RESNET_ARCH, seed=0)
    y = np.random.default_rng(1).standard_normal((2, 3072 + 128 * 11 + 77)).astype(np.float32)
    x = oracle.unfold_windows(y.astype(np.float64), 3072, 128)[:12]
    c = np.random.default_rng(99).standard_normal((2, 3072 + 1000 * 15 + 77)).astype(np.float32)
    calib = oracle.unfold_windows(c.astype(np.float64), 3072, 1000)[:16]
    ref = oracle.net_forward(params, RESNET_ARCH, x)
    plain = oracle.net_forward_quant(params, RESNET_ARCH, x, "fp8")
    corr = oracle.net_forward_quant(params, RESNET_ARCH, x, "fp8", calib=calib)
    assert np.abs(plain - ref).max() > 0.1
    assert np.abs(corr - ref).max() < 0.08
