"""GPU: streaming server.  Streamed results equal the offline path over the
same data; a stream's results are identical alone and in a mix; admission
respects the HBM budget."""
import numpy as np
import pytest
import torch

from synth import TINY_ARCH, make_params
from synth.noise import coloured_noise
from tests.gpu_util import banner, dev, need_gpu

pytestmark = pytest.mark.gpu
FS = 2048


def run_stream(server, sid_data, chunk_plan, rng=None):
    """Push each stream's data in the planned chunk sizes, ticking at random
    points; return {sid: (logits, integrated)}."""
    from paper_2403_18661_amd.stream import Collector
    col = Collector()
    pos = {sid: 0 for sid in sid_data}
    rng = rng or np.random.default_rng(0)
    active = set(sid_data)
    while active:
        for sid in list(active):
            x = sid_data[sid]
            n = chunk_plan(rng)
            if pos[sid] >= x.shape[1]:
                active.discard(sid)
                continue
            server.push(sid, x[:, pos[sid]:pos[sid] + n])
            pos[sid] += n
        if rng.random() < 0.7:
            server.tick()
            for sid in sid_data:
                col.take(server, sid)
    server.tick()
    server.tick()
    for sid in sid_data:
        col.take(server, sid)
    return {sid: col.arrays(sid) for sid in sid_data}


def test_stream_equals_offline():
    P = need_gpu()
    from paper_2403_18661_amd.pipeline import OfflinePath, PathConfig
    from paper_2403_18661_amd.stream import Server
    banner("stream vs offline")
    params = make_params(TINY_ARCH, seed=31)
    net = P.Net(TINY_ARCH, params, "f32")
    x = coloured_noise(FS * 84, seed=32)
    srv = Server(net, max_streams=4, hbm_budget=4 << 30)
    sid = srv.admit()
    out = run_stream(srv, {sid: x}, lambda r: FS)[sid]
    path = OfflinePath(net, x.shape[1], PathConfig(psd_len=64 * FS))
    path.run(torch.from_numpy(x).cuda())
    lg, ig = path.logits.cpu().numpy(), path.integrated.cpu().numpy()
    assert len(out[0]) > 100 and len(out[1]) > 80
    n = len(out[0])
    assert n <= len(lg)
    np.testing.assert_allclose(out[0], lg[:n], atol=1e-4)
    m = len(out[1])
    np.testing.assert_allclose(out[1], ig[:m], atol=1e-4)


def test_stream_long_equals_offline():
    """150 s in 1 s chunks: the raw ring (about 85 s) is compacted several
    times, and every later PSD and whitening block must still see its data."""
    P = need_gpu()
    from paper_2403_18661_amd.pipeline import OfflinePath, PathConfig
    from paper_2403_18661_amd.stream import Server
    banner("stream vs offline, 150 s (raw ring compaction)")
    params = make_params(TINY_ARCH, seed=35)
    net = P.Net(TINY_ARCH, params, "f32")
    x = coloured_noise(FS * 150, seed=36)
    srv = Server(net, max_streams=2, hbm_budget=4 << 30)
    sid = srv.admit()
    out = run_stream(srv, {sid: x}, lambda r: FS, np.random.default_rng(3))[sid]
    path = OfflinePath(net, x.shape[1], PathConfig(psd_len=64 * FS))
    path.run(torch.from_numpy(x).cuda())
    lg, ig = path.logits.cpu().numpy(), path.integrated.cpu().numpy()
    n, m = len(out[0]), len(out[1])
    assert n > 16 * 80 and n <= len(lg)
    np.testing.assert_allclose(out[0], lg[:n], atol=1e-4)
    np.testing.assert_allclose(out[1], ig[:m], atol=1e-4)


def test_alone_equals_in_the_mix():
    P = need_gpu()
    from paper_2403_18661_amd.stream import Server
    banner("stream alone vs mix")
    params = make_params(TINY_ARCH, seed=33)
    net = P.Net(TINY_ARCH, params, "bf16")
    xs = [coloured_noise(FS * 80, seed=40 + k) for k in range(3)]
    srv = Server(net, max_streams=4, hbm_budget=4 << 30)
    a = srv.admit()
    alone = run_stream(srv, {a: xs[0]}, lambda r: FS, np.random.default_rng(1))[a]
    srv.release(a)
    ids = [srv.admit() for _ in range(3)]
    mixed = run_stream(srv, dict(zip(ids, xs)), lambda r: int(r.integers(300, 5000)), np.random.default_rng(2))
    got = mixed[ids[0]]
    assert len(alone[0]) > 50
    np.testing.assert_array_equal(got[0], alone[0])
    np.testing.assert_array_equal(got[1], alone[1])
    st = srv.stats()
    assert st["samples"] > 0 and st["p99_ms"] > 0


def test_budget_admission_and_release():
    P = need_gpu()
    from paper_2403_18661_amd.stream import Server
    net = P.Net(TINY_ARCH, make_params(TINY_ARCH, seed=1), "bf16")
    probe = Server(net, max_streams=8, hbm_budget=4 << 30)
    per, shared = probe.stream_bytes, probe.shared_bytes
    probe.close()
    srv = Server(net, max_streams=8, hbm_budget=shared + 2 * per)
    a, b = srv.admit(), srv.admit()
    with pytest.raises(P.AframeError, match="EBUDGET"):
        srv.admit()
    srv.release(a)
    c = srv.admit()
    assert c == a
    with pytest.raises(P.AframeError, match="EINVAL"):
        srv.push(b, np.zeros((2, 10 ** 6)))          # longer than max_chunk


def test_pushes_from_another_thread_during_ticks():
    # a producer thread pushes chunks of three streams at random moments while
    # this thread ticks and polls (chunks that arrive while a tick runs join a
    # later tick); every stream's results equal its run alone, bit for bit
    P = need_gpu()
    import threading
    import time
    from paper_2403_18661_amd.stream import Collector, Server
    banner("stream pushes from a second thread during ticks")
    params = make_params(TINY_ARCH, seed=37)
    net = P.Net(TINY_ARCH, params, "bf16")
    xs = [coloured_noise(FS * 76, seed=60 + k) for k in range(3)]
    srv = Server(net, max_streams=4, hbm_budget=4 << 30)
    alone = []
    for x in xs:
        a = srv.admit()
        alone.append(run_stream(srv, {a: x}, lambda r: FS, np.random.default_rng(5))[a])
        srv.release(a)
    ids = [srv.admit() for _ in range(3)]
    done = threading.Event()

    def producer():
        rng = np.random.default_rng(9)
        pos = [0, 0, 0]
        while any(pos[k] < xs[k].shape[1] for k in range(3)):
            k = int(rng.integers(3))
            if pos[k] >= xs[k].shape[1]:
                continue
            n = int(rng.integers(500, 4000))
            srv.push(ids[k], xs[k][:, pos[k]:pos[k] + n])
            pos[k] += n
            time.sleep(float(rng.uniform(0, 0.002)))
        done.set()

    th = threading.Thread(target=producer)
    col = Collector()
    th.start()
    ticks = 0
    while not done.is_set():
        srv.tick()
        ticks += 1
        for sid in ids:
            col.take(srv, sid)
    th.join()
    for _ in range(40):     # drain what is still pending (a tick takes at most max_tick per stream)
        srv.tick()
    for sid in ids:
        col.take(srv, sid)
    assert ticks > 10
    for k, sid in enumerate(ids):
        lg, ig = col.arrays(sid)
        assert len(lg) == len(alone[k][0]) > 50
        np.testing.assert_array_equal(lg, alone[k][0])
        np.testing.assert_array_equal(ig, alone[k][1])
