"""The paper's own form of the scoring network, forward pass in FP64 (oracle).

The paper replaces BatchNorm with GroupNorm throughout its 1D ResNet34 (Sec. II)
and uses convolutions of kernel length 3 with global pooling (Sec. IX).  Unlike
eval-mode BatchNorm, GroupNorm normalises with statistics of the window being
scored, so it cannot be folded into the convolutions.

GroupNorm with G groups: the C channels split into G runs of C/G consecutive
channels; for each window and group, mu and var are the mean and the biased
variance over the group's channels and all time samples, and channel c maps
    v -> gamma_c (v - mu) / sqrt(var + eps) + beta_c,   eps = 1e-5.

    stem  : conv k, stride s0, 'same' zero padding, no bias -> GN -> ReLU [-> maxpool k3 s2 p1]
    block : y = ReLU( GN2(conv2( ReLU(GN1(conv1(x))) )) + skip ),
            skip = x, or GN(conv 1x1 stride 2 (x)) when the shape changes
    head  : global average pool over time -> fully connected -> 1 logit

Pins (tests/test_oracle_gn.py): group_norm == brute-force loops; G = C equals
torch's instance_norm and G = 1 its layer_norm over (C, L); unit moments of the
normalised groups; invariance to an affine map of the input; the whole forward
== a torch.nn float64 model built from GroupNorm modules.
"""
import numpy as np

from .net import conv1d, maxpool3s2

GN_EPS = 1e-5


def group_norm(x, gamma, beta, groups, eps=GN_EPS):
    """x [B, C, L] -> GroupNorm(groups) with per-channel affine gamma, beta [C]."""
    B, C, L = x.shape
    xg = x.reshape(B, groups, (C // groups) * L)
    mu = xg.mean(axis=2, keepdims=True)
    var = ((xg - mu) ** 2).mean(axis=2, keepdims=True)
    y = ((xg - mu) / np.sqrt(var + eps)).reshape(B, C, L)
    return y * gamma[None, :, None] + beta[None, :, None]


def net_forward_gn(params, arch, x, return_features=False):
    """x [B, in_ch, window] float64 -> logits [B] (float64)."""
    relu = lambda v: np.maximum(v, 0.0)

    def conv(h, name, stride):
        w = params[name + ".w"]
        return conv1d(h, w, np.zeros(w.shape[0]), stride)

    def gn(h, name):
        return group_norm(h, params[name + ".gamma"], params[name + ".beta"], arch.groups)

    h = relu(gn(conv(x, "stem.conv", arch.stem_stride), "stem.bn"))
    if arch.stem_pool:
        h = maxpool3s2(h)
    for pre, _, _, stride, proj in arch.block_list():
        r = relu(gn(conv(h, pre + ".conv1", stride), pre + ".bn1"))
        r = gn(conv(r, pre + ".conv2", 1), pre + ".bn2")
        skip = gn(conv(h, pre + ".proj", stride), pre + ".projbn") if proj else h
        h = relu(r + skip)
    g = h.mean(axis=2)
    logits = g @ params["fc.w"][0] + params["fc.b"][0]
    return (logits, g) if return_features else logits
