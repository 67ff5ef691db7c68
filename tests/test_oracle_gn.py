"""Pins of the GroupNorm network oracle (oracle/net_gn.py)."""
import numpy as np
import pytest
import torch

import oracle
from oracle.net_gn import group_norm
from synth import GN_ARCH, GN_NARROW_ARCH, TINY_GN_ARCH, make_params


def test_group_norm_matches_brute_force_loops():
    rng = np.random.default_rng(0)
    B, C, L, G = 2, 8, 5, 4
    x = rng.standard_normal((B, C, L)) * 3 + 1
    gamma, beta = rng.standard_normal(C), rng.standard_normal(C)
    ref = np.zeros_like(x)
    cpg = C // G
    for b in range(B):
        for g in range(G):
            vals = [x[b, c, t] for c in range(g * cpg, (g + 1) * cpg) for t in range(L)]
            n = len(vals)
            mu = sum(vals) / n
            var = sum((v - mu) ** 2 for v in vals) / n
            for c in range(g * cpg, (g + 1) * cpg):
                for t in range(L):
                    ref[b, c, t] = gamma[c] * (x[b, c, t] - mu) / (var + 1e-5) ** 0.5 + beta[c]
    np.testing.assert_allclose(group_norm(x, gamma, beta, G), ref, rtol=1e-12, atol=1e-12)


def test_group_norm_special_cases_are_instance_and_layer_norm():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 6, 40))
    gamma, beta = rng.uniform(0.5, 1.5, 6), rng.standard_normal(6)
    inst = torch.nn.functional.instance_norm(torch.from_numpy(x), weight=torch.from_numpy(gamma),
                                             bias=torch.from_numpy(beta), eps=1e-5).numpy()
    np.testing.assert_allclose(group_norm(x, gamma, beta, 6), inst, atol=1e-12)
    lay = torch.nn.functional.layer_norm(torch.from_numpy(x), (6, 40), eps=1e-5).numpy()
    lay = lay * gamma[None, :, None] + beta[None, :, None]
    np.testing.assert_allclose(group_norm(x, gamma, beta, 1), lay, atol=1e-12)


def test_normalised_groups_have_unit_moments_and_affine_invariance():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 16, 100)) * 50 + 7
    y = group_norm(x, np.ones(16), np.zeros(16), 4).reshape(2, 4, -1)
    np.testing.assert_allclose(y.mean(axis=2), 0.0, atol=1e-12)
    np.testing.assert_allclose(y.var(axis=2), 1.0, rtol=1e-8)       # eps / var ~ 4e-9
    g, b = rng.standard_normal(16), rng.standard_normal(16)
    np.testing.assert_allclose(group_norm(3 * x - 11, g, b, 4), group_norm(x, g, b, 4), rtol=1e-7, atol=1e-7)


class TorchBlock(torch.nn.Module):
    def __init__(self, c_in, c_out, stride, proj, k, G):
        super().__init__()
        self.conv1 = torch.nn.Conv1d(c_in, c_out, k, stride, k // 2, bias=False)
        self.gn1 = torch.nn.GroupNorm(G, c_out)
        self.conv2 = torch.nn.Conv1d(c_out, c_out, k, 1, k // 2, bias=False)
        self.gn2 = torch.nn.GroupNorm(G, c_out)
        self.proj = torch.nn.Sequential(torch.nn.Conv1d(c_in, c_out, 1, stride, bias=False),
                                        torch.nn.GroupNorm(G, c_out)) if proj else None

    def forward(self, x):
        r = torch.relu(self.gn1(self.conv1(x)))
        r = self.gn2(self.conv2(r))
        return torch.relu(r + (self.proj(x) if self.proj is not None else x))


def torch_gn_model(arch, params):
    """A torch.nn float64 GroupNorm ResNet-1D assembled independently of the oracle."""
    k, G = arch.kernel, arch.groups
    stem = [torch.nn.Conv1d(arch.in_ch, arch.stem_ch, k, arch.stem_stride, k // 2, bias=False),
            torch.nn.GroupNorm(G, arch.stem_ch), torch.nn.ReLU()]
    if arch.stem_pool:
        stem.append(torch.nn.MaxPool1d(3, 2, 1))
    blocks = [TorchBlock(ci, co, s, p, k, G) for _, ci, co, s, p in arch.block_list()]
    fc = torch.nn.Linear(arch.widths[-1], 1)
    model = torch.nn.ModuleDict({"stem": torch.nn.Sequential(*stem), "blocks": torch.nn.Sequential(*blocks),
                                 "fc": fc}).double().eval()

    def set_gn(gn, pre):
        gn.weight.copy_(torch.from_numpy(params[pre + ".gamma"]))
        gn.bias.copy_(torch.from_numpy(params[pre + ".beta"]))

    with torch.no_grad():
        model["stem"][0].weight.copy_(torch.from_numpy(params["stem.conv.w"]))
        set_gn(model["stem"][1], "stem.bn")
        for blk, (pre, _, _, _, p) in zip(model["blocks"], arch.block_list()):
            blk.conv1.weight.copy_(torch.from_numpy(params[pre + ".conv1.w"])); set_gn(blk.gn1, pre + ".bn1")
            blk.conv2.weight.copy_(torch.from_numpy(params[pre + ".conv2.w"])); set_gn(blk.gn2, pre + ".bn2")
            if p:
                blk.proj[0].weight.copy_(torch.from_numpy(params[pre + ".proj.w"])); set_gn(blk.proj[1], pre + ".projbn")
        fc.weight.copy_(torch.from_numpy(params["fc.w"])); fc.bias.copy_(torch.from_numpy(params["fc.b"]))

    def run(x):
        with torch.no_grad():
            h = model["blocks"](model["stem"](torch.from_numpy(x)))
            return model["fc"](h.mean(dim=2))[:, 0].numpy()
    return run


@pytest.mark.parametrize("arch", [TINY_GN_ARCH, GN_NARROW_ARCH, GN_ARCH],
                         ids=["tiny-gn", "resnet34-gn-narrow", "resnet34-gn"])
def test_forward_matches_torch_gn_model(arch):
    params = make_params(arch, seed=5)
    x = np.random.default_rng(6).standard_normal((2, arch.in_ch, arch.window))
    np.testing.assert_allclose(oracle.net_forward_gn(params, arch, x), torch_gn_model(arch, params)(x),
                               rtol=1e-9, atol=1e-9)


def test_gn_params_hold_no_running_statistics():
    p = make_params(TINY_GN_ARCH, seed=0)
    assert not any(k.endswith((".mean", ".var")) for k in p)
    # conv weights, then per norm gamma and beta, then fc
    n_conv = 2 * 32 * 3 + (32 * 32 * 3) * 4 + (64 * 32 * 3 + 64 * 64 * 3 + 64 * 32)
    n_norm = 2 * (32 + 32 * 4 + 64 * 3)
    assert sum(v.size for v in p.values()) == n_conv + n_norm + 64 + 1
