"""Architectures and seeded random parameters of the 1D residual scoring network.

The paper's network is a ResNet34 variant with 1D convolutions (Sec. II); the
main workloads use a folded-BatchNorm variant with kernel 7, and the paper's own
form (GroupNorm in place of BatchNorm, Sec. II; kernel length 3, Sec. IX) is
`norm="gn"`.  Trained weights are not available, so parameters are drawn from
a seed:

* conv weights: He-normal, std sqrt(2 / (C_in k)); convs carry no bias;
* BatchNorm (eps 1e-5): gamma ~ U(0.9, 1.1) except the last BN of each residual
  branch, gamma ~ U(0.2, 0.3) (a damped residual branch keeps activations O(1)
  through 16 blocks without running the network to calibrate statistics);
  beta ~ N(0, 0.02^2), running mean ~ N(0, 0.05^2), running var ~ U(0.8, 1.25);
* GroupNorm (eps 1e-5): per-channel gamma and beta drawn like BatchNorm's
  (the damped range for the last norm of each residual branch);
* FC: He-normal weight (fan-in C), bias 0.

Parameters are returned as an ordered dict name -> float64 array; the order is
the order in which the layers run.
"""
from collections import OrderedDict
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class NetArch:
    name: str
    in_ch: int
    stem_ch: int
    kernel: int
    stem_stride: int
    stem_pool: bool          # max-pool k3 s2 p1 after the stem ReLU
    widths: tuple
    blocks: tuple
    window: int = 3072
    norm: str = "bn"         # "bn" (folded BatchNorm) or "gn" (GroupNorm)
    groups: int = 0          # GroupNorm groups per layer

    def block_list(self):
        """Yield (prefix, c_in, c_out, stride, has_proj) for every BasicBlock."""
        c_in = self.stem_ch
        for s, (w, nb) in enumerate(zip(self.widths, self.blocks)):
            for b in range(nb):
                stride = 2 if (b == 0 and s > 0) else 1
                proj = stride != 1 or c_in != w
                yield f"s{s}.b{b}", c_in, w, stride, proj
                c_in = w


TINY_ARCH = NetArch("tiny", in_ch=2, stem_ch=16, kernel=7, stem_stride=1,
                    stem_pool=False, widths=(16,), blocks=(2,))
RESNET_ARCH = NetArch("resnet", in_ch=2, stem_ch=32, kernel=7, stem_stride=2,
                      stem_pool=True, widths=(32, 64, 128, 256), blocks=(3, 4, 6, 3))
# the paper's form: GroupNorm, kernel length 3, ResNet34 at its standard
# widths (64-channel stem, stages of 64, 128, 256 and 512 channels)
GN_ARCH = NetArch("resnet34-gn", in_ch=2, stem_ch=64, kernel=3, stem_stride=2, stem_pool=True,
                  widths=(64, 128, 256, 512), blocks=(3, 4, 6, 3), norm="gn", groups=8)
# the same depth at half the widths (the widths of the BatchNorm network)
GN_NARROW_ARCH = NetArch("resnet34-gn-narrow", in_ch=2, stem_ch=32, kernel=3, stem_stride=2, stem_pool=True,
                         widths=(32, 64, 128, 256), blocks=(3, 4, 6, 3), norm="gn", groups=8)
TINY_GN_ARCH = NetArch("tiny-gn", in_ch=2, stem_ch=32, kernel=3, stem_stride=2, stem_pool=True,
                       widths=(32, 64), blocks=(2, 1), window=512, norm="gn", groups=8)


def _bn(rng, c, damped=False):
    lo, hi = (0.2, 0.3) if damped else (0.9, 1.1)
    return {
        "gamma": rng.uniform(lo, hi, c),
        "beta": 0.02 * rng.standard_normal(c),
        "mean": 0.05 * rng.standard_normal(c),
        "var": rng.uniform(0.8, 1.25, c),
    }


def make_params(arch, seed=0):
    rng = np.random.default_rng(seed)
    k = arch.kernel
    p = OrderedDict()

    def conv(name, c_out, c_in, kk):
        p[name + ".w"] = np.sqrt(2.0 / (c_in * kk)) * rng.standard_normal((c_out, c_in, kk))

    def bn(name, c, damped=False):
        for key, v in _bn(rng, c, damped).items():
            if arch.norm == "gn" and key in ("mean", "var"):
                continue                      # GroupNorm has no running statistics
            p[f"{name}.{key}"] = v

    conv("stem.conv", arch.stem_ch, arch.in_ch, k)
    bn("stem.bn", arch.stem_ch)
    for pre, c_in, c_out, stride, proj in arch.block_list():
        conv(pre + ".conv1", c_out, c_in, k)
        bn(pre + ".bn1", c_out)
        conv(pre + ".conv2", c_out, c_out, k)
        bn(pre + ".bn2", c_out, damped=True)
        if proj:
            conv(pre + ".proj", c_out, c_in, 1)
            bn(pre + ".projbn", c_out)
    c_last = arch.widths[-1]
    p["fc.w"] = np.sqrt(2.0 / c_last) * rng.standard_normal((1, c_last))
    p["fc.b"] = np.zeros(1)
    return p
