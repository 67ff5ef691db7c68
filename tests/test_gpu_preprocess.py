"""GPU parity: Welch PSD, whitening and integration against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from synth import analytic_psd, coloured_noise
from tests.gpu_util import banner, dev, need_gpu, rel_l2

pytestmark = pytest.mark.gpu
FS = 2048.0
PRESCALE = 1e21


@pytest.mark.parametrize("nperseg,n,n_ch,dtype", [(4096, 32768, 2, "f64"), (512, 5000, 3, "f64"),
                                                  (4096, 32768, 2, "f32"), (256, 256, 1, "f64")])
def test_psd_single(nperseg, n, n_ch, dtype):
    P = need_gpu()
    banner(f"psd single nperseg={nperseg} n={n} n_ch={n_ch} {dtype}")
    x = coloured_noise(n, seed=1, n_ch=n_ch)
    if dtype == "f32":
        xs = (x * PRESCALE).astype(np.float32)
        got = P.psd_estimate(dev(xs), FS, 1.0, nperseg=nperseg).cpu().numpy()[0]
        ref = oracle.welch_psd(xs.astype(np.float64), FS, nperseg, nperseg // 2)
    else:
        got = P.psd_estimate(dev(x), FS, PRESCALE, nperseg=nperseg).cpu().numpy()[0]
        ref = oracle.welch_psd(x * PRESCALE, FS, nperseg, nperseg // 2)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12 * ref.max())


def test_psd_rolling():
    P = need_gpu()
    banner("psd rolling 3 hops")
    x = coloured_noise(2048 * 40, seed=2)
    got = P.psd_estimate(dev(x), FS, PRESCALE, psd_len=2048 * 16, psd_hop=2048 * 8, n_psd=3).cpu().numpy()
    ref = oracle.welch_psd_rolling(x * PRESCALE, FS, 2048 * 16, 2048 * 8, 3)
    np.testing.assert_allclose(got, ref, rtol=1e-10)


def test_psd_rejects_bad_args():
    P = need_gpu()
    x = dev(coloured_noise(8192, seed=0))
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.psd_estimate(x, FS, PRESCALE, nperseg=3000)
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.psd_estimate(x, FS, PRESCALE, psd_len=4096, psd_hop=1000, n_psd=2)


@pytest.mark.parametrize("n,n_ch", [(32768, 2), (2048 * 9 + 517, 1), (20000, 3)])
def test_whiten_same_psd(n, n_ch):
    # both sides whiten with the analytic PSD sampled on the Welch grid
    P = need_gpu()
    banner(f"whiten analytic psd n={n} n_ch={n_ch}")
    x = coloured_noise(n, seed=3, n_ch=n_ch)
    f = np.arange(2049) * FS / 4096
    psd = np.broadcast_to(analytic_psd(f) * PRESCALE ** 2, (n_ch, 2049)).copy()
    got = P.whiten(dev(x), dev(psd[None]), FS, PRESCALE).cpu().numpy()
    ref = oracle.whiten(x * PRESCALE, psd, FS)
    assert got.shape == ref.shape
    for c in range(n_ch):
        assert rel_l2(got[c], ref[c]) < 1e-5


def test_whiten_c1_end_to_end_psd():
    # plain path, tiny config: 16 s, PSD from the same 16 s, crop 0.5 s per edge
    P = need_gpu()
    banner("whiten C1 (16 s, own Welch PSD)")
    x = coloured_noise(32768, seed=0)
    xd = dev(x)
    psd = P.psd_estimate(xd, FS, PRESCALE)
    y = P.whiten(xd, psd, FS, PRESCALE).cpu().numpy()
    ref = oracle.whiten(x, oracle.welch_psd(x, FS), FS)   # scale invariance: no prescale needed
    assert y.shape == (2, 30720)
    for c in range(2):
        assert rel_l2(y[c], ref[c]) < 1e-5


def test_whiten_f32_input():
    P = need_gpu()
    banner("whiten f32 prescaled input")
    x = (coloured_noise(24576, seed=4) * PRESCALE).astype(np.float32)
    xd = dev(x)
    psd = P.psd_estimate(xd, FS, 1.0)
    y = P.whiten(xd, psd, FS, 1.0).cpu().numpy()
    x64 = x.astype(np.float64)
    ref = oracle.whiten(x64, oracle.welch_psd(x64, FS), FS)
    for c in range(2):
        assert rel_l2(y[c], ref[c]) < 1e-5


def test_whiten_piecewise_hops_and_ragged_tail():
    # rolling background: hop j whitens [n0 + j*hop, n0 + (j+1)*hop) with the PSD of
    # the psd_len samples ending M before it; ragged last hop
    P = need_gpu()
    banner("whiten piecewise 4 hops")
    psd_len, hop, M = 2048 * 8, 2048 * 4, 1024
    n0 = psd_len + M
    n_out = 3 * hop + 5000
    n = n0 + n_out + M
    x = coloured_noise(n, seed=5)
    xd = dev(x)
    psd = P.psd_estimate(xd, FS, PRESCALE, psd_len=psd_len, psd_hop=hop, n_psd=4)
    y = P.whiten(xd, psd, FS, PRESCALE, psd_hop=hop, out_start=n0, n_out=n_out).cpu().numpy()
    psd_ref = oracle.welch_psd_rolling(x, FS, psd_len, hop, 4)
    ref = oracle.whiten_piecewise(x, psd_ref, FS, n0, n_out, hop)
    for c in range(2):
        assert rel_l2(y[c], ref[c]) < 1e-5
        for j in range(4):       # each hop individually
            lo, hi = j * hop, min((j + 1) * hop, n_out)
            assert rel_l2(y[c, lo:hi], ref[c, lo:hi]) < 1e-5


def test_whiten_variance_band_fraction():
    P = need_gpu()
    banner("whiten variance 256 s")
    x = coloured_noise(2048 * 256, seed=6)
    f = np.arange(2049) * FS / 4096
    psd = np.broadcast_to(analytic_psd(f) * PRESCALE ** 2, (2, 2049)).copy()
    y = P.whiten(dev(x), dev(psd[None]), FS, PRESCALE).cpu().numpy()
    np.testing.assert_allclose(y.var(axis=1), 0.96875, rtol=0.02)


def test_whiten_rejects_short_context():
    P = need_gpu()
    x = dev(coloured_noise(8192, seed=0))
    psd = P.psd_estimate(x, FS, PRESCALE)
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.whiten(x, psd, FS, PRESCALE, out_start=1000, n_out=100)


@pytest.mark.parametrize("n,width", [(217, 16), (5000, 16), (10, 16), (16, 16), (33, 1)])
def test_integrate(n, width):
    P = need_gpu()
    p = np.random.default_rng(n).standard_normal(n).astype(np.float32)
    got = P.integrate(dev(p), width).cpu().numpy()
    ref = oracle.integrate(p.astype(np.float64), width)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6)


def test_whiten_response_apply_split():
    """af_whiten_response + af_whiten_apply = af_whiten bit for bit (rolling
    PSDs, FP64 input); undersized buffers are rejected before any launch."""
    P = need_gpu()
    banner("whiten split response/apply")
    import torch
    fs = int(FS)
    x = coloured_noise(fs * 96, seed=77)
    xd = dev(x)
    hop = 8 * fs
    n_psd = 3
    psd = P.psd_estimate(xd, FS, PRESCALE, psd_len=64 * fs, psd_hop=hop, n_psd=n_psd)
    M = fs // 2
    out_start = 64 * fs + M
    n_out = xd.shape[1] - out_start - M
    ref = P.whiten(xd, psd, FS, PRESCALE, hop, out_start=out_start, n_out=n_out)
    resp = P.whiten_response(psd, FS)
    got = P.whiten_apply(xd, resp, n_psd, FS, PRESCALE, hop, out_start=out_start, n_out=n_out)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    small = resp[: resp.numel() // 2]
    with pytest.raises(P.AframeError):
        P.whiten_apply(xd, small, n_psd, FS, PRESCALE, hop, out_start=out_start, n_out=n_out)
    with pytest.raises(P.AframeError):
        P.whiten_response(psd, FS, out=small)


def test_integrate_carry_streams_equal_the_batch():
    # chunks of every size (shorter than the carry, single samples, long runs)
    # through one carry give the batch values bit for bit from the width-th
    # output on
    P = need_gpu()
    import torch
    banner("integrate with carry")
    for width in (16, 4, 2048):
        n = 5000
        p = dev(np.random.default_rng(width).standard_normal(n).astype(np.float32))
        ref = P.integrate(p, width).cpu().numpy()
        carry = torch.zeros(width - 1, dtype=torch.float32, device="cuda")
        outs, i = [], 0
        for size in (5, 1, 37, 300, 1, 2100, 0, 2556):
            outs.append(P.integrate(p[i:i + size], width, carry=carry).cpu().numpy())
            i += size
        assert i == n
        got = np.concatenate(outs)
        assert got.shape == (n,)
        np.testing.assert_array_equal(got[width - 1:], ref)
        np.testing.assert_array_equal(carry.cpu().numpy(), p[n - width + 1:].cpu().numpy())
    one = dev(np.arange(7, dtype=np.float32))
    np.testing.assert_array_equal(P.integrate(one, 1, carry=torch.zeros(0, device="cuda")).cpu().numpy(),
                                  np.arange(7, dtype=np.float32))


def test_whiten_apply_checks_the_response_it_is_given():
    # a response built for another filter length, fewer PSDs or another
    # channel count, or one no af_whiten_response call filled, is rejected
    P = need_gpu()
    import torch
    fs = int(FS)
    xd = dev(coloured_noise(fs * 40, seed=78))
    psd = P.psd_estimate(xd, FS, PRESCALE)
    resp = P.whiten_response(psd, FS, fduration=1.0)
    ok = P.whiten_apply(xd, resp, 1, FS, PRESCALE, fduration=1.0)
    assert ok.shape[1] == xd.shape[1] - fs
    with pytest.raises(P.AframeError, match="taps"):
        P.whiten_apply(xd, resp, 1, FS, PRESCALE, fduration=0.5)
    roomy = torch.empty(2 * resp.numel(), dtype=torch.uint8, device="cuda")   # room for two PSDs, filled with one
    P.whiten_response(psd, FS, out=roomy)
    with pytest.raises(P.AframeError, match="PSDs"):
        P.whiten_apply(xd, roomy, 2, FS, PRESCALE, psd_hop=8 * fs, fduration=1.0)
    with pytest.raises(P.AframeError, match="too small"):
        P.whiten_apply(xd, resp, 2, FS, PRESCALE, psd_hop=8 * fs, fduration=1.0)
    with pytest.raises(P.AframeError, match="af_whiten_response"):
        P.whiten_apply(xd, torch.zeros_like(resp), 1, FS, PRESCALE, fduration=1.0)


def test_psd_and_whitening_captured_after_init_replay_equal():
    # af_init builds the constant tables up front, so the PSD and whitening
    # calls can be captured in a graph; every replay equals the direct calls
    P = need_gpu()
    import torch
    from paper_2403_18661_amd.timeslides import Graph
    banner("psd + whiten graph capture")
    P.check(P.lib().af_init())
    fs = int(FS)
    xd = dev(coloured_noise(fs * 24, seed=79))
    ws_p = torch.empty(P.lib().af_psd_workspace_bytes(2, 4096, 2048, xd.shape[1], 0, 1), dtype=torch.uint8,
                       device="cuda")
    ws_w = torch.empty(P.lib().af_whiten_workspace_bytes(2, 4096, 1), dtype=torch.uint8, device="cuda")
    psd_ref = P.psd_estimate(xd, FS, PRESCALE, ws=ws_p)
    y_ref = P.whiten(xd, psd_ref, FS, PRESCALE, ws=ws_w)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    psd = torch.empty_like(psd_ref)
    y = torch.empty_like(y_ref)
    g = Graph(s)
    with g:   # every buffer exists beforehand: nothing is allocated during the capture
        P.psd_estimate(xd, FS, PRESCALE, out=psd, ws=ws_p, stream=s)
        P.whiten(xd, psd, FS, PRESCALE, out=y, ws=ws_w, stream=s)
    for rep in range(3):
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.launch()
        s.synchronize()
        assert torch.equal(psd, psd_ref) and torch.equal(y, y_ref)
        _ = (xd * 2).sum().item()        # unrelated eager work between replays
    g.close()
