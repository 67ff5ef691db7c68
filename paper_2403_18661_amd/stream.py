"""Streaming server binding (af_server_*) and a real-time arrival driver.

The server keeps per-stream state on the device and scores the new windows
of all streams together in each tick; see include/aframe_mi.h.
"""
import ctypes
import time

import numpy as np

from ._lib import ServerConfig, check, lib


def default_config(**overrides):
    cfg = ServerConfig()
    lib().af_server_default_config(ctypes.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


class Server:
    def __init__(self, net, **cfg):
        self.net = net            # keeps the net alive as long as the server
        self.cfg = default_config(**cfg)
        h = ctypes.c_void_p()
        check(lib().af_server_create(net._h, ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h
        self._cap = 1 << 16

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().af_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream_bytes(self):
        return lib().af_server_stream_bytes(self._h)

    @property
    def shared_bytes(self):
        return lib().af_server_shared_bytes(self._h)

    def admit(self):
        sid = ctypes.c_int64()
        check(lib().af_server_admit(self._h, ctypes.byref(sid)))
        return sid.value

    def release(self, sid):
        check(lib().af_server_release(self._h, sid))

    def push(self, sid, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        check(lib().af_server_push(self._h, sid, x.ctypes.data_as(ctypes.c_void_p), x.shape[-1]))

    def tick(self):
        n = ctypes.c_int64()
        check(lib().af_server_tick(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, sid):
        """-> (first_logit_index, logits, first_integrated_index, integrated)"""
        lg = np.empty(self._cap, np.float32)
        ig = np.empty(self._cap, np.float32)
        nl, fl, ni, fi = (ctypes.c_int64() for _ in range(4))
        check(lib().af_server_poll(self._h, sid, lg.ctypes.data_as(ctypes.c_void_p), self._cap, ctypes.byref(nl),
                                   ctypes.byref(fl), ig.ctypes.data_as(ctypes.c_void_p), self._cap,
                                   ctypes.byref(ni), ctypes.byref(fi)))
        return fl.value, lg[:nl.value].copy(), fi.value, ig[:ni.value].copy()

    def stats(self, reset=False):
        p50, p99 = ctypes.c_double(), ctypes.c_double()
        n, w = ctypes.c_int64(), ctypes.c_int64()
        check(lib().af_server_stats(self._h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(n), ctypes.byref(w),
                                    int(reset)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "samples": n.value, "windows": w.value}


class Collector:
    """Accumulates polled results per stream into contiguous arrays."""

    def __init__(self):
        self.logits, self.integ = {}, {}

    def take(self, server, sid):
        fl, lg, fi, ig = server.poll(sid)
        for store, first, vals in ((self.logits, fl, lg), (self.integ, fi, ig)):
            if len(vals):
                cur = store.setdefault(sid, [])
                n = sum(len(v) for v in cur)
                assert first == n, "results must arrive in order"
                cur.append(vals)

    def arrays(self, sid):
        cat = lambda d: np.concatenate(d.get(sid, [np.zeros(0, np.float32)]))
        return cat(self.logits), cat(self.integ)


def run_realtime(server, data, seconds, fs=2048, chunk_s=1.0, prefill_s=66.0, seed=0, log=None):
    """Drive `server` with Poisson-jittered 1 s chunks per stream in real time.

    data: list of [n_ch, n] float64 arrays, one per stream (already admitted
    streams 0..S-1).  Each stream is first pre-filled with `prefill_s` seconds
    (pushed and ticked at once) so that its PSD background and first windows
    exist; latency statistics are reset after the pre-fill.  Then for
    `seconds` of wall time each stream's next chunk arrives after an
    exponential gap of mean chunk_s; the loop pushes chunks as their arrival
    times pass and runs a tick whenever anything is pending.
    """
    rng = np.random.default_rng(seed)
    S = len(data)
    n_chunk = int(chunk_s * fs)
    pos = [0] * S
    for i in range(S):
        n_pre = int(prefill_s * fs)
        for a in range(0, n_pre, n_chunk):
            server.push(i, data[i][:, a:a + n_chunk])
        pos[i] = n_pre
    # a tick consumes at most max_tick samples per stream: drain the pre-fill
    for _ in range(int(prefill_s * fs) // int(server.cfg.max_tick) + 3):
        server.tick()
        for i in range(S):
            server.poll(i)
    server.stats(reset=True)
    t0 = time.perf_counter()
    nxt = [t0 + rng.exponential(chunk_s) for _ in range(S)]
    ticks = 0
    last_log = t0
    while True:
        now = time.perf_counter()
        if now - t0 > seconds:
            break
        pushed = 0
        for i in range(S):
            while nxt[i] <= now and pos[i] + n_chunk <= data[i].shape[1]:
                server.push(i, data[i][:, pos[i]:pos[i] + n_chunk])
                pos[i] += n_chunk
                nxt[i] += rng.exponential(chunk_s)
                pushed += 1
        if pushed:
            server.tick()
            ticks += 1
            for i in range(S):
                server.poll(i)
        else:
            time.sleep(max(0.0, min(min(nxt) - time.perf_counter(), 0.002)))
        if log and now - last_log > 10:
            log(f"stream run: {now - t0:.0f} s, {ticks} ticks")
            last_log = now
    elapsed = time.perf_counter() - t0
    st = server.stats()
    st.update({"streams": S, "seconds": elapsed, "ticks": ticks, "windows_per_s": st["windows"] / elapsed})
    return st
