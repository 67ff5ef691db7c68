"""Pins for oracle.net (1D residual network forward pass)."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from oracle.net import maxpool3s2, folded_layers
from synth import TINY_ARCH, RESNET_ARCH, make_params


def brute_conv(x, w, b, stride):
    B, C, L = x.shape
    O, _, k = w.shape
    pad = (k - 1) // 2
    L_out = (L + 2 * pad - k) // stride + 1
    out = np.zeros((B, O, L_out))
    for bi, o, t in itertools.product(range(B), range(O), range(L_out)):
        acc = b[o]
        for c in range(C):
            for j in range(k):
                s = t * stride + j - pad
                if 0 <= s < L:
                    acc += w[o, c, j] * x[bi, c, s]
        out[bi, o, t] = acc
    return out


@pytest.mark.parametrize("L,stride,k,C,O", [(13, 1, 7, 3, 2), (14, 2, 7, 2, 3), (9, 2, 1, 4, 2), (5, 1, 7, 1, 1)])
def test_conv1d_brute(L, stride, k, C, O):
    rng = np.random.default_rng(L * 7 + k)
    x = rng.standard_normal((2, C, L))
    w = rng.standard_normal((O, C, k))
    b = rng.standard_normal(O)
    np.testing.assert_allclose(oracle.conv1d(x, w, b, stride), brute_conv(x, w, b, stride), atol=1e-12)


def test_conv1d_matches_torch_float64():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 16, 200))
    w = rng.standard_normal((32, 16, 7))
    b = rng.standard_normal(32)
    for s in (1, 2):
        ref = torch.nn.functional.conv1d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b),
                                         stride=s, padding=3).numpy()
        np.testing.assert_allclose(oracle.conv1d(x, w, b, s), ref, atol=1e-11)


def test_maxpool_matches_torch():
    x = np.random.default_rng(1).standard_normal((2, 3, 20))
    ref = torch.nn.functional.max_pool1d(torch.from_numpy(x), 3, 2, 1).numpy()
    np.testing.assert_array_equal(maxpool3s2(x), ref)


def test_bn_fold_equals_conv_then_bn():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 8, 50))
    w = rng.standard_normal((6, 8, 7))
    g, be, mu, var = rng.uniform(0.5, 2, 6), rng.standard_normal(6), rng.standard_normal(6), rng.uniform(0.5, 2, 6)
    wf, bf = oracle.fold_bn(w, g, be, mu, var)
    bn = torch.nn.BatchNorm1d(6, eps=1e-5).double().eval()
    with torch.no_grad():
        bn.weight.copy_(torch.from_numpy(g)); bn.bias.copy_(torch.from_numpy(be))
        bn.running_mean.copy_(torch.from_numpy(mu)); bn.running_var.copy_(torch.from_numpy(var))
        ref = bn(torch.nn.functional.conv1d(torch.from_numpy(x), torch.from_numpy(w), padding=3)).numpy()
    np.testing.assert_allclose(oracle.conv1d(x, wf, bf), ref, atol=1e-11)


class TorchBlock(torch.nn.Module):
    def __init__(self, c_in, c_out, stride, proj):
        super().__init__()
        self.conv1 = torch.nn.Conv1d(c_in, c_out, 7, stride, 3, bias=False)
        self.bn1 = torch.nn.BatchNorm1d(c_out)
        self.conv2 = torch.nn.Conv1d(c_out, c_out, 7, 1, 3, bias=False)
        self.bn2 = torch.nn.BatchNorm1d(c_out)
        self.proj = torch.nn.Sequential(torch.nn.Conv1d(c_in, c_out, 1, stride, bias=False),
                                        torch.nn.BatchNorm1d(c_out)) if proj else None

    def forward(self, x):
        r = torch.relu(self.bn1(self.conv1(x)))
        r = self.bn2(self.conv2(r))
        return torch.relu(r + (self.proj(x) if self.proj is not None else x))


def torch_model(arch, params):
    """A torch.nn float64 ResNet-1D assembled independently of the oracle."""
    stem = [torch.nn.Conv1d(arch.in_ch, arch.stem_ch, 7, arch.stem_stride, 3, bias=False),
            torch.nn.BatchNorm1d(arch.stem_ch), torch.nn.ReLU()]
    if arch.stem_pool:
        stem.append(torch.nn.MaxPool1d(3, 2, 1))
    blocks = [TorchBlock(ci, co, s, p) for _, ci, co, s, p in arch.block_list()]
    fc = torch.nn.Linear(arch.widths[-1], 1)
    model = torch.nn.ModuleDict({"stem": torch.nn.Sequential(*stem), "blocks": torch.nn.Sequential(*blocks), "fc": fc})
    model = model.double().eval()

    def set_bn(bn, pre):
        bn.weight.copy_(torch.from_numpy(params[pre + ".gamma"])); bn.bias.copy_(torch.from_numpy(params[pre + ".beta"]))
        bn.running_mean.copy_(torch.from_numpy(params[pre + ".mean"])); bn.running_var.copy_(torch.from_numpy(params[pre + ".var"]))

    with torch.no_grad():
        model["stem"][0].weight.copy_(torch.from_numpy(params["stem.conv.w"]))
        set_bn(model["stem"][1], "stem.bn")
        for blk, (pre, _, _, _, p) in zip(model["blocks"], arch.block_list()):
            blk.conv1.weight.copy_(torch.from_numpy(params[pre + ".conv1.w"])); set_bn(blk.bn1, pre + ".bn1")
            blk.conv2.weight.copy_(torch.from_numpy(params[pre + ".conv2.w"])); set_bn(blk.bn2, pre + ".bn2")
            if p:
                blk.proj[0].weight.copy_(torch.from_numpy(params[pre + ".proj.w"])); set_bn(blk.proj[1], pre + ".projbn")
        fc.weight.copy_(torch.from_numpy(params["fc.w"])); fc.bias.copy_(torch.from_numpy(params["fc.b"]))

    def run(x):
        with torch.no_grad():
            h = model["blocks"](model["stem"](torch.from_numpy(x)))
            return model["fc"](h.mean(dim=2))[:, 0].numpy()
    run.model = model
    return run


@pytest.mark.parametrize("arch", [TINY_ARCH, RESNET_ARCH], ids=lambda a: a.name)
def test_forward_matches_torch_model(arch):
    params = make_params(arch, seed=3)
    x = np.random.default_rng(4).standard_normal((2, 2, 3072))
    ref = torch_model(arch, params)(x)
    np.testing.assert_allclose(oracle.net_forward(params, arch, x), ref, rtol=1e-10, atol=1e-10)


def _macs(arch):
    L = arch.window
    L_stem = L // arch.stem_stride
    macs = L_stem * arch.stem_ch * arch.in_ch * arch.kernel
    L = L_stem // 2 if arch.stem_pool else L_stem
    for _, ci, co, s, p in arch.block_list():
        Lo = L // s
        macs += Lo * co * ci * arch.kernel + Lo * co * co * arch.kernel + (Lo * co * ci if p else 0)
        L = Lo
    return macs + arch.widths[-1]


def test_mac_counts_match_golden():
    golden = {}
    for line in open(__file__.replace("test_oracle_net.py", "golden/arch_macs.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            golden[k] = int(v)
    assert _macs(TINY_ARCH) == golden["tiny"]
    assert _macs(RESNET_ARCH) == golden["resnet"]


@pytest.mark.parametrize("prec,tol", [("bf16", 0.03), ("fp8", 0.1)])
def test_quant_emulation_within_precision_bound(prec, tol):
    arch = TINY_ARCH
    params = make_params(arch, seed=0)
    x = np.random.default_rng(5).standard_normal((4, 2, 3072)).astype(np.float32).astype(np.float64)
    ref = oracle.net_forward(params, arch, x)
    q = oracle.net_forward_quant(params, arch, x, prec)
    assert np.max(np.abs(q - ref)) < tol
    assert np.max(np.abs(q - ref)) > 0


def test_fp8_conv_is_exact_when_operands_sit_on_the_grid():
    # operands already on the E4M3 grid with max |.| = 448 give unit scales, so
    # quantisation is the identity and the emulated conv equals the plain one
    from oracle.net import _quant_conv
    rng = np.random.default_rng(6)
    grid = oracle.e4m3_round(rng.uniform(-448, 448, 4000))
    h = np.abs(rng.choice(grid, size=(2, 16, 40)))
    h[0, 0, 0] = h[1, 3, 7] = 448.0
    w = rng.choice(grid, size=(8, 16, 7))
    w[:, 0, 0] = 448.0
    b = rng.standard_normal(8)
    acc, deq = _quant_conv(h, w, b, 1, "fp8")
    np.testing.assert_array_equal(deq, 1.0)
    np.testing.assert_allclose(acc, oracle.conv1d(h, w, np.zeros(8)), rtol=1e-15)
    # halving the input halves the activation scale and nothing else
    acc2, deq2 = _quant_conv(h / 2, w, b, 1, "fp8")
    np.testing.assert_array_equal(acc2, acc)
    np.testing.assert_array_equal(deq2, 0.5)
