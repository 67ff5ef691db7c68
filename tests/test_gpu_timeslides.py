"""GPU parity: timeslide background scoring (af_score_timeslides) against the
oracle applied to explicitly shifted segments."""
import numpy as np
import pytest

import oracle
from synth import TINY_ARCH, make_params
from tests.gpu_util import banner, dev, need_gpu

pytestmark = pytest.mark.gpu


def oracle_timeslides(params, arch, y, seg_off, seg_len, shifts, stride):
    out = []
    for o, L in zip(seg_off, seg_len):
        seg = y[:, o:o + L].astype(np.float64)
        for k in shifts:
            w = oracle.unfold_windows(seg, arch.window, stride, np.array([0, k % L]), L)
            out.append(oracle.net_forward(params, arch, w) if len(w) else np.zeros(0))
    return np.concatenate(out)


@pytest.mark.parametrize("prec,tol", [("f32", 2e-5), ("bf16", 3e-2)])
def test_timeslides_vs_oracle(prec, tol):
    P = need_gpu()
    banner(f"timeslides {prec}")
    params = make_params(TINY_ARCH, seed=11)
    rng = np.random.default_rng(12)
    seg_off, seg_len = [100, 9000, 14500], [8000, 5000, 2000]    # the last one is shorter than a window
    n = 16600
    y = rng.standard_normal((2, n)).astype(np.float32)
    shifts = [2048, 4096, 6144 + 3]
    net = P.Net(TINY_ARCH, params, prec)
    got = P.score_timeslides(net, dev(y), seg_off, seg_len, shifts, stride=1024, batch=7).cpu().numpy()
    ref = oracle_timeslides(params, TINY_ARCH, y, seg_off, seg_len, shifts, 1024)
    assert got.shape == ref.shape == (P.timeslide_n_windows(seg_len, 3, 3072, 1024),)
    assert np.abs(got - ref).max() < tol


def test_zero_shift_equals_plain_windows():
    P = need_gpu()
    params = make_params(TINY_ARCH, seed=13)
    y = np.random.default_rng(14).standard_normal((2, 12000)).astype(np.float32)
    net = P.Net(TINY_ARCH, params, "f32")
    ts = P.score_timeslides(net, dev(y), [1000], [10000], [0, 10000], stride=512).cpu().numpy()
    plain = net.score_windows(dev(y[:, 1000:11000].copy()), 512).cpu().numpy()
    nw = len(plain)
    np.testing.assert_array_equal(ts[:nw], plain)
    np.testing.assert_array_equal(ts[nw:], plain)     # a full-length shift is no shift


def test_segments_shorter_than_a_window_give_no_windows():
    # every segment shorter than a window: no windows, an empty result and no
    # launch, in both the layer and the whole-network path
    P = need_gpu()
    y = dev(np.zeros((2, 6000), np.float32))
    assert P.timeslide_n_windows([3071, 2000], 2, 3072, 2048) == 0
    for prec in ("f32", "bf16"):
        net = P.Net(TINY_ARCH, make_params(TINY_ARCH, seed=1), prec)
        out = P.score_timeslides(net, y, [0, 3500], [3071, 2000], [2048, 4096])
        assert out.numel() == 0


def test_rejects_segment_outside_series():
    P = need_gpu()
    net = P.Net(TINY_ARCH, make_params(TINY_ARCH, seed=1), "f32")
    y = dev(np.zeros((2, 5000), np.float32))
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.score_timeslides(net, y, [1000], [4500], [2048])


def test_prepared_graph_replays_match_direct_call():
    # the captured graph, replayed several times with eager work in between,
    # gives the direct call's logits every time
    P = need_gpu()
    import torch
    from paper_2403_18661_amd.timeslides import TimeslidePlan
    banner("timeslide graph replay")
    params = make_params(TINY_ARCH, seed=15)
    y = dev(np.random.default_rng(16).standard_normal((2, 20000)).astype(np.float32))
    net = P.Net(TINY_ARCH, params, "bf16")
    seg_off, seg_len, shifts = [0, 9000], [9000, 11000], [2048 * k for k in range(1, 6)]
    direct = P.score_timeslides(net, y, seg_off, seg_len, shifts, stride=1024).cpu().numpy()
    plan = TimeslidePlan(net, y, seg_off, seg_len, shifts, stride=1024, graph=True)
    for rep in range(3):
        plan.logits.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run()
        plan.stream.synchronize()
        np.testing.assert_array_equal(plan.logits[:plan.n_windows].cpu().numpy(), direct)
        _ = (y * 2).sum().item()          # unrelated eager work between replays


def test_graph_replays_after_a_tile_switch():
    # a graph captured on the layer path keeps the weight image and tile it
    # captured; switching a layer's tile afterwards leaves its replays equal
    # to the direct call
    P = need_gpu()
    import torch
    from paper_2403_18661_amd.timeslides import TimeslidePlan
    banner("graph replay after set_tile")
    params = make_params(TINY_ARCH, seed=17)
    y = dev(np.random.default_rng(18).standard_normal((2, 20000)).astype(np.float32))
    net = P.Net(TINY_ARCH, params, "f32")
    seg_off, seg_len, shifts = [0, 9000], [9000, 11000], [2048 * k for k in range(1, 4)]
    direct = P.score_timeslides(net, y, seg_off, seg_len, shifts, stride=1024).cpu().numpy()
    plan = TimeslidePlan(net, y, seg_off, seg_len, shifts, stride=1024, graph=True)
    tiles = net.tiles()
    switched = 0
    for layer, (_, _, n_cand, chosen) in enumerate(tiles, start=1):
        if n_cand > 1:
            net.set_tile(layer, (chosen + 1) % n_cand)
            switched += 1
    assert switched > 0
    for rep in range(2):
        plan.logits.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run()
        plan.stream.synchronize()
        np.testing.assert_array_equal(plan.logits[:plan.n_windows].cpu().numpy(), direct)
    np.testing.assert_array_equal(P.score_timeslides(net, y, seg_off, seg_len, shifts, stride=1024).cpu().numpy(),
                                  direct)


def test_full_day_sampled_windows():
    # the benchmark's timeslide workload at full size (24 h in 40 lognormal
    # segments, 100 slides of k x 1 s, 1 Hz windows, the autotuned whole-network
    # kernel in a hipGraph) on a seeded stand-in for the whitened series;
    # sampled windows, wrap-crossing ones included, against the oracle
    P = need_gpu()
    import torch
    from paper_2403_18661_amd.timeslides import TimeslidePlan
    from synth import lognormal_segments
    banner("timeslides, full day, sampled windows")
    fs, stride, W = 2048, 2048, TINY_ARCH.window
    seg_len = [int(d) * fs - 133120 for d in lognormal_segments(seed=0)]
    seg_len = [L for L in seg_len if L >= W]
    seg_off = list(np.cumsum([0] + seg_len[:-1]))
    y = np.random.default_rng(15).standard_normal((2, sum(seg_len)), dtype=np.float32)
    shifts = [k * fs for k in range(1, 101)]
    params = make_params(TINY_ARCH, seed=0)
    net = P.Net(TINY_ARCH, params, "bf16")
    net.autotune(batch=8192)
    plan = TimeslidePlan(net, dev(y), seg_off, seg_len, shifts, stride=stride, graph=True)
    plan.run()
    plan.stream.synchronize()
    got = plan.logits[:plan.n_windows].cpu().numpy()
    assert plan.n_windows == P.timeslide_n_windows(seg_len, len(shifts), W, stride) > 8_000_000
    nw = [(L - W) // stride + 1 for L in seg_len]
    base = np.cumsum([0] + [n * len(shifts) for n in nw[:-1]])
    rng = np.random.default_rng(16)
    picks = [(0, 0, 0), (len(seg_len) - 1, 99, nw[-1] - 1)]
    for s in rng.choice(len(seg_len), 6, replace=False):
        k = int(rng.integers(100))
        # the last window of a slide: its L1 part wraps past the segment's end
        picks += [(int(s), k, nw[s] - 1), (int(s), k, int(rng.integers(nw[s])))]
    wins, idx = [], []
    for s, k, i in picks:
        o, L = seg_off[s], seg_len[s]
        t = i * stride + np.arange(W)
        wins.append(np.stack([y[0, o + t], y[1, o + (t + shifts[k]) % L]]).astype(np.float64))
        idx.append(base[s] + k * nw[s] + i)
    wins = np.stack(wins)
    ref = oracle.net_forward(params, TINY_ARCH, wins)
    emu = oracle.net_forward_quant(params, TINY_ARCH, wins, "bf16")
    err, err_emu = np.abs(got[idx] - ref).max(), np.abs(got[idx] - emu).max()
    print(f"{len(idx)} sampled windows of {plan.n_windows}: |d| vs FP64 {err:.2e}, vs BF16 emulation {err_emu:.2e}")
    assert err < 3e-2 and err_emu < 2e-5
    del plan
    torch.cuda.empty_cache()
