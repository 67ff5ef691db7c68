"""Pins of where net_forward_quant rounds (oracle/net.py).

The BF16 modes round at fixed points: the stem output, every conv operand,
the inner activation of a block, the projection, the block output.  A network
of one channel, 1x1 kernels and a one-sample window reduces the forward pass
to scalar arithmetic, and inputs on or just off the BF16 grid make each
rounding point change the logit.  Expected values are worked out by hand
below with u = 2^-8 (half the BF16 spacing 2^-7 on [1, 2); the spacing is 4u
on [2, 4) and 8u on [4, 8)); ties go to the even mantissa.  Moving any one
rounding point (skipping it, or rounding to the other precision) changes at
least one of these values.
"""
from collections import OrderedDict

import numpy as np

import oracle
from synth.params import NetArch

U = 2.0 ** -8
ONE_BLOCK = NetArch("pin1", in_ch=1, stem_ch=1, kernel=1, stem_stride=1, stem_pool=False,
                    widths=(1,), blocks=(1,), window=1)                       # identity skip
TWO_STAGES = NetArch("pin2", in_ch=1, stem_ch=1, kernel=1, stem_stride=1, stem_pool=False,
                     widths=(1, 1), blocks=(1, 1), window=1)                  # second block projects


def scalar_net(arch, ws, a1, a2, p=None):
    """Parameters whose BatchNorms fold to scale 1 and bias 0 exactly
    (gamma = sqrt(var + eps) computed the way the fold computes it)."""
    par = OrderedDict()

    def conv(name, v):
        par[name + ".w"] = np.array([[[v]]])

    def bn(name):
        par[name + ".gamma"] = np.array([np.sqrt(1.0 + 1e-5)])
        par[name + ".beta"] = np.zeros(1)
        par[name + ".mean"] = np.zeros(1)
        par[name + ".var"] = np.ones(1)

    conv("stem.conv", ws); bn("stem.bn")
    for pre, _, _, _, proj in arch.block_list():
        conv(pre + ".conv1", a1); bn(pre + ".bn1")
        conv(pre + ".conv2", a2); bn(pre + ".bn2")
        if proj:
            conv(pre + ".proj", p); bn(pre + ".projbn")
    par["fc.w"] = np.ones((1, 1))
    par["fc.b"] = np.zeros(1)
    return par


def logit(arch, x, prec, **w):
    par = scalar_net(arch, **w)
    folded = oracle.net.folded_layers(par, arch)
    assert all(v[0].ravel()[0] == par[k + ".w"].ravel()[0] and v[1][0] == 0.0 for k, v in folded.items())
    return oracle.net_forward_quant(par, arch, np.array([[[x]]]), prec)[0]


# ---- 'bf16': BF16 operands, every stored tensor BF16 ------------------------
def test_bf16_inner_activation_and_block_output_rounding():
    # stem  (1+3u)(1+u) = 1+4u+3u^2 -> stored BF16: 1+4u
    # conv1 (1+4u)(1+2u) = 1+6u+8u^2 -> stored BF16 (inner activation): 1+6u
    # conv2 weight 1+u -> BF16 1 (tie to even); 1+6u + skip 1+4u = 2+10u, a tie
    #       between 2+8u (even) and 2+12u -> 2+8u
    # (unrounded inner activation: 2+10u+8u^2 -> 2+12u; stem stored FP32:
    #  2+10u+3u^2 -> 2+12u; unrounded weight: 2+11u+6u^2 -> 2+12u; block output
    #  not stored: 2+10u)
    assert logit(ONE_BLOCK, 1 + 3 * U, "bf16", ws=1 + U, a1=1 + 2 * U, a2=1 + U) == 2 + 8 * U


def test_bf16_block_output_rounds_after_the_residual_add():
    # stem 1+4u; conv1 weight 1+u -> 1: inner 1+4u; conv2 (1+4u)(1+2u) = 1+6u+8u^2
    # + skip 1+4u = 2+10u+8u^2, just above the tie -> 2+12u.  Rounding the conv2
    # output before the add gives 1+6u + 1+4u = 2+10u -> 2+8u instead.
    assert logit(ONE_BLOCK, 1 + 3 * U, "bf16", ws=1 + U, a1=1 + U, a2=1 + 2 * U) == 2 + 12 * U


def test_bf16_projection_is_stored_before_the_add():
    # stem 1+4u; block 1 (weights 1+u -> 1): inner 1+4u, output 2+8u.
    # block 2: inner 2+8u; projection (2+8u)(1+2u) = 2+12u+16u^2 -> stored BF16
    # 2+12u; 2+8u + 2+12u = 4+20u, a tie between 4+16u (even) and 4+24u -> 4+16u.
    # (projection not stored: 4+20u+16u^2 -> 4+24u)
    assert logit(TWO_STAGES, 1 + 3 * U, "bf16", ws=1 + U, a1=1 + U, a2=1 + U, p=1 + 2 * U) == 4 + 16 * U


# ---- 'bf16f': BF16 operands, stored tensors FP32 -----------------------------
def test_bf16f_stem_and_block_output_stay_fp32():
    # stem (1+u)^2 = 1+2u+u^2 (FP32-exact, kept); conv1 operand BF16 1+2u, weight
    # 1+u -> 1: inner 1+2u; conv2 1+2u + skip 1+2u+u^2 = 2+4u+u^2 (kept in FP32).
    # (stem or block output stored BF16: 2+4u; weights unrounded: 2+7u+5u^2)
    assert logit(ONE_BLOCK, 1 + U, "bf16f", ws=1 + U, a1=1 + U, a2=1 + U) == 2 + 4 * U + U * U


def test_bf16f_rounds_the_first_conv_operand():
    # stem 1+u; conv1 operand BF16(1+u) = 1 (tie), times 1+2u: inner 1+2u;
    # conv2 (weight 1) 1+2u + skip 1+u = 2+3u.  (operand unrounded: inner
    # 1+3u+2u^2, whose BF16 operand 1+4u gives 2+5u)
    assert logit(ONE_BLOCK, 1 + U, "bf16f", ws=1.0, a1=1 + 2 * U, a2=1 + U) == 2 + 3 * U


def test_bf16f_rounds_the_inner_activation_as_the_second_conv_operand():
    # stem 1+2u+u^2; conv1 BF16 operand 1+2u times 1+2u: inner 1+4u+4u^2 (FP32);
    # conv2 operand BF16 1+4u (weight 1) + skip 1+2u+u^2 = 2+6u+u^2.
    # (operand unrounded: 2+6u+5u^2)
    assert logit(ONE_BLOCK, 1 + U, "bf16f", ws=1 + U, a1=1 + 2 * U, a2=1 + U) == 2 + 6 * U + U * U


def test_bf16f_projection_operand_rounds_and_its_output_stays_fp32():
    # stem 1+2u+u^2; block 1 output 2+4u+u^2 (as above).  Block 2: conv1 operand
    # BF16 2+4u (weight 1): inner 2+4u; projection operand BF16 2+4u times 1+2u
    # = 2+8u+8u^2 (kept FP32); conv2 2+4u + 2+8u+8u^2 = 4+12u+8u^2.
    # (projection stored BF16: 4+12u; its operand unrounded: 4+12u+9u^2+2u^3)
    assert logit(TWO_STAGES, 1 + U, "bf16f", ws=1 + U, a1=1 + U, a2=1 + U, p=1 + 2 * U) == 4 + 12 * U + 8 * U * U


def test_values_used_above_sit_where_the_derivations_say():
    from oracle.quant import bf16_round as B
    assert B(1 + U) == 1.0 and B(1 + 3 * U) == 1 + 4 * U and B(1 + 2 * U) == 1 + 2 * U
    assert B(2 + 10 * U) == 2 + 8 * U and B(4 + 20 * U) == 4 + 16 * U
    assert np.float32(1 + 4 * U + 3 * U * U) == 1 + 4 * U + 3 * U * U   # FP32-exact products
