"""GPU parity of the GroupNorm, kernel-3 network (af_net_create_gn) against the
FP64 oracle (oracle/net_gn.py)."""
import dataclasses

import numpy as np
import pytest

import oracle
from synth import GN_ARCH, GN_NARROW_ARCH, TINY_GN_ARCH, make_params
from tests.gpu_util import banner, dev, need_gpu

pytestmark = pytest.mark.gpu

# logit tolerances against the FP64 oracle, per precision
TOL = {"f32": 1e-3, "bf16f": 3e-2}


def series(n, seed, n_ch=2):
    return np.random.default_rng(seed).standard_normal((n_ch, n)).astype(np.float32)


def oracle_logits(params, arch, y, stride, nw, shifts=None, wrap=0):
    w = oracle.unfold_windows(y.astype(np.float64), arch.window, stride, shifts, wrap)[:nw]
    return oracle.net_forward_gn(params, arch, w)


# a 480-sample window gives a 240-row stem, which the one-pass stem kernel does
# not take (rows per thread block must be even): the two-kernel stem runs
TINY480_GN_ARCH = dataclasses.replace(TINY_GN_ARCH, name="tiny480-gn", window=480)
# the widest stages the GroupNorm net takes (1024 channels), on a short window
WIDE_GN_ARCH = dataclasses.replace(TINY_GN_ARCH, name="wide-gn", stem_ch=64, widths=(64, 1024), blocks=(1, 2))


@pytest.mark.parametrize("arch,prec,nw", [(TINY_GN_ARCH, "f32", 37), (TINY_GN_ARCH, "bf16f", 37),
                                          (TINY480_GN_ARCH, "f32", 9), (WIDE_GN_ARCH, "f32", 11),
                                          (WIDE_GN_ARCH, "bf16f", 11),
                                          (GN_NARROW_ARCH, "f32", 5), (GN_NARROW_ARCH, "bf16f", 5),
                                          (GN_ARCH, "f32", 5), (GN_ARCH, "bf16f", 5)],
                         ids=["tiny-f32", "tiny-bf16f", "tiny480-f32", "wide-f32", "wide-bf16f",
                              "resnet34-narrow-f32", "resnet34-narrow-bf16f", "resnet34-f32", "resnet34-bf16f"])
def test_gn_net_matches_oracle(arch, prec, nw):
    P = need_gpu()
    banner(f"gn net {arch.name} {prec} nw={nw}")
    params = make_params(arch, seed=51)
    stride = 160
    y = series(arch.window + stride * (nw - 1) + 7, seed=52)
    got = P.Net(arch, params, prec).score_windows(dev(y), stride, nw).cpu().numpy()
    ref = oracle_logits(params, arch, y, stride, nw)
    err = np.abs(got - ref).max()
    print(f"{arch.name} {prec}: max |d logit| {err:.2e} (logit spread {ref.std():.2f})")
    assert err < TOL[prec]
    if prec == "f32":
        assert err < 1e-4 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("prec", ["f32", "bf16f"])
def test_gn_edge_cases(prec):
    # no windows, exactly one window (the series is one window long), and a
    # window past the end rejected, at the standard widths
    P = need_gpu()
    banner(f"gn edge cases {prec}")
    params = make_params(GN_ARCH, seed=64)
    net = P.Net(GN_ARCH, params, prec)
    y = series(GN_ARCH.window, seed=65)
    assert net.score_windows(dev(y), 128, 0).numel() == 0
    one = net.score_windows(dev(y), 128, 1).cpu().numpy()
    ref = oracle_logits(params, GN_ARCH, y, 128, 1)
    assert np.abs(one - ref).max() < TOL[prec]
    with pytest.raises(P.AframeError, match="EINVAL"):
        net.score_windows(dev(y), 128, 2)


def test_gn_statistics_are_per_window():
    # a window's logit does not depend on the batch it is scored in
    P = need_gpu()
    banner("gn batch independence")
    params = make_params(TINY_GN_ARCH, seed=53)
    y = dev(series(512 + 64 * 40, seed=54))
    net = P.Net(TINY_GN_ARCH, params, "f32")
    full = net.score_windows(y, 64, batch=1024).cpu().numpy()
    for b in (1, 3, 16):
        assert np.array_equal(net.score_windows(y, 64, batch=b).cpu().numpy(), full)


def test_gn_shifts_wrap_and_timeslides():
    P = need_gpu()
    banner("gn shifts+wrap, timeslides")
    params = make_params(TINY_GN_ARCH, seed=55)
    n = 512 * 6
    y = series(n, seed=56)
    shifts = [0, 1000]
    net = P.Net(TINY_GN_ARCH, params, "f32")
    got = net.score_windows(dev(y), 256, 9, shifts=shifts, wrap=n).cpu().numpy()
    ref = oracle_logits(params, TINY_GN_ARCH, y, 256, 9, np.array(shifts), n)
    assert np.abs(got - ref).max() < 1e-4
    seg_off, seg_len, slides = [10, 1500, 2600], [1400, 1000, 400], [128, 512 + 3]
    got = P.score_timeslides(net, dev(y), seg_off, seg_len, slides, stride=96, batch=5).cpu().numpy()
    ref = []
    for o, L in zip(seg_off, seg_len):
        seg = y[:, o:o + L].astype(np.float64)
        for k in slides:
            w = oracle.unfold_windows(seg, 512, 96, np.array([0, k % L]), L)
            ref.append(oracle.net_forward_gn(params, TINY_GN_ARCH, w) if len(w) else np.zeros(0))
    ref = np.concatenate(ref)
    assert got.shape == ref.shape and np.abs(got - ref).max() < 1e-4


@pytest.mark.parametrize("prec", ["f32", "bf16f"])
def test_every_gn_tile_candidate_same_logits(prec):
    # every tile shape of every k3 / 1x1 layer gives the default's logits bit for bit
    P = need_gpu()
    banner(f"gn tile candidates {prec}")
    params = make_params(GN_ARCH, seed=57)
    y = dev(series(3072 + 128 * 3, seed=58))
    net = P.Net(GN_ARCH, params, prec)
    ref = net.score_windows(y, 128, batch=4).cpu().numpy()
    tried = 0
    for layer, (_, _, n_cand, chosen) in enumerate(net.tiles(), start=1):
        for c in range(n_cand):
            if c == chosen:
                continue
            net.set_tile(layer, c)
            got = net.score_windows(y, 128, batch=4).cpu().numpy()
            assert np.array_equal(got, ref), f"layer {layer} candidate {c}: max|d| {np.abs(got - ref).max():.3e}"
            tried += 1
        net.set_tile(layer, chosen)
    print(f"{prec}: {tried} alternative tiles, all identical")


def test_gn_rejects_unsupported_forms():
    P = need_gpu()
    params = make_params(TINY_GN_ARCH, seed=59)
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.Net(TINY_GN_ARCH, params, "bf16")                       # BF16 activations: not for GroupNorm
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.Net(dataclasses.replace(TINY_GN_ARCH, groups=3), params, "f32")   # 3 does not divide 32
    k7 = dataclasses.replace(TINY_GN_ARCH, kernel=7)
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.Net(k7, make_params(k7, seed=59), "f32")
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.Net(TINY_GN_ARCH, np.zeros(10), "f32")                   # params too short


def test_gn_stream_equals_offline():
    # the streaming server scores a GroupNorm net's windows as the offline path does
    P = need_gpu()
    import torch
    from paper_2403_18661_amd.pipeline import OfflinePath, PathConfig
    from paper_2403_18661_amd.stream import Server
    from synth.noise import coloured_noise
    from tests.test_gpu_stream import run_stream
    banner("gn stream vs offline")
    fs = 2048
    params = make_params(GN_ARCH, seed=60)
    net = P.Net(GN_ARCH, params, "f32")
    x = coloured_noise(fs * 84, seed=61)
    srv = Server(net, max_streams=2, hbm_budget=4 << 30)
    sid = srv.admit()
    out = run_stream(srv, {sid: x}, lambda r: fs)[sid]
    path = OfflinePath(net, x.shape[1], PathConfig(psd_len=64 * fs))
    path.run(torch.from_numpy(x).cuda())
    lg, ig = path.logits.cpu().numpy(), path.integrated.cpu().numpy()
    n, m = len(out[0]), len(out[1])
    assert n > 100 and m > 80 and n <= len(lg)
    np.testing.assert_allclose(out[0], lg[:n], atol=1e-5)
    np.testing.assert_allclose(out[1], ig[:m], atol=1e-5)


def test_gn_timeslide_graph_replays_match_direct_call():
    # the GroupNorm launches capture into the timeslide graph: every replay,
    # with eager work in between, gives the direct call's logits
    P = need_gpu()
    import torch
    from paper_2403_18661_amd.timeslides import TimeslidePlan
    banner("gn timeslide graph replay")
    params = make_params(TINY_GN_ARCH, seed=62)
    y = dev(series(6000, seed=63))
    net = P.Net(TINY_GN_ARCH, params, "f32")
    seg_off, seg_len, shifts = [0, 2500], [2500, 3500], [256 * k for k in range(1, 5)]
    direct = P.score_timeslides(net, y, seg_off, seg_len, shifts, stride=128).cpu().numpy()
    plan = TimeslidePlan(net, y, seg_off, seg_len, shifts, stride=128, graph=True)
    assert plan.n_windows == len(direct) > 0
    for _ in range(3):
        plan.logits.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run()
        plan.stream.synchronize()
        np.testing.assert_array_equal(plan.logits[:plan.n_windows].cpu().numpy(), direct)
        _ = (y * 2).sum().item()
