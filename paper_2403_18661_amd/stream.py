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
    exist; latency statistics are reset after the pre-fill.  Then, for
    `seconds` of wall time, a producer thread pushes each stream's next chunk
    at its arrival time (exponential gaps of mean chunk_s), also while a tick
    runs, and this thread ticks whenever chunks are pending.  The server
    stamps a chunk when it is pushed, i.e. at its arrival, so the latency
    includes any wait behind a tick that was already running.
    """
    import threading
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
    arrivals = []            # (time, stream) in arrival order
    for i in range(S):
        t = t0 + rng.exponential(chunk_s)
        k = pos[i]
        while t < t0 + seconds and k + n_chunk <= data[i].shape[1]:
            arrivals.append((t, i, k))
            k += n_chunk
            t += rng.exponential(chunk_s)
    arrivals.sort()
    pending = threading.Semaphore(0)
    stop = threading.Event()

    def producer():
        for t, i, k in arrivals:
            wait = t - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            server.push(i, data[i][:, k:k + n_chunk])
            pending.release()
        stop.set()

    th = threading.Thread(target=producer, daemon=True)
    th.start()
    ticks = 0
    last_log = t0
    while True:
        if not pending.acquire(timeout=0.05):
            if stop.is_set():
                break
            continue
        while pending.acquire(blocking=False):   # every chunk pushed so far joins this tick
            pass
        server.tick()
        ticks += 1
        for i in range(S):
            server.poll(i)
        now = time.perf_counter()
        if log and now - last_log > 10:
            log(f"stream run: {now - t0:.0f} s, {ticks} ticks")
            last_log = now
    th.join()
    server.tick()
    for i in range(S):
        server.poll(i)
    elapsed = time.perf_counter() - t0
    st = server.stats()
    st.update({"streams": S, "seconds": elapsed, "ticks": ticks, "windows_per_s": st["windows"] / elapsed,
               "latency_from": "chunk arrival (pushed by a producer thread at its scheduled time)"})
    return st
