"""Timeslide background scoring as one replayable graph.

The work table ((segment, slide) -> window range) is copied to the device once
(af_timeslide_prepare); scoring every window of every slide is then one
enqueue (with the whole-network kernel: one persistent launch), captured once
in a hipGraph and replayed per run.
"""
import ctypes

import torch

from . import _i64, _ptr, _stream, _workspace, check, lib, timeslide_n_windows


class Graph:
    """Capture of library calls on a non-default stream (af_graph_*)."""

    def __init__(self, stream):
        self.stream = stream
        self._h = None

    def __enter__(self):
        check(lib().af_graph_begin(_stream(self.stream)))
        return self

    def __exit__(self, exc_type, exc, tb):
        h = ctypes.c_void_p()
        rc = lib().af_graph_end(_stream(self.stream), ctypes.byref(h))
        if exc_type is None:
            check(rc)
            self._h = h
        return False

    def launch(self, stream=None):
        check(lib().af_graph_launch(self._h, _stream(stream if stream is not None else self.stream)))

    def close(self):
        if self._h is not None and self._h.value:
            lib().af_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TimeslidePlan:
    def __init__(self, net, y, seg_off, seg_len, shifts, stride=2048, batch=4096, graph=True):
        self.net, self.y, self.stride = net, y, stride
        n_ch, n = y.shape
        self.so, self.pso = _i64(seg_off)
        self.sl, self.psl = _i64(seg_len)
        self.sh, self.psh = _i64(shifts)
        self.n_windows = timeslide_n_windows(self.sl, len(self.sh), net.window, stride)
        self.logits = torch.empty(max(self.n_windows, 1), dtype=torch.float32, device=y.device)
        self.ws = _workspace(lib().af_timeslide_workspace_bytes(net._h, len(self.so), len(self.sh),
                                                                max(1, min(batch, self.n_windows))), y.device)
        self.stream = torch.cuda.Stream()
        check(lib().af_timeslide_prepare(net._h, self.pso, self.psl, len(self.so), self.psh, len(self.sh), stride, n,
                                         _ptr(self.ws), self.ws.numel(), _stream(self.stream)))
        self.graph = None
        if graph:
            self.graph = Graph(self.stream)
            with self.graph:
                self._enqueue(self.stream)

    def _enqueue(self, stream):
        n_ch, n = self.y.shape
        check(lib().af_score_timeslides_prepared(self.net._h, _ptr(self.y), n_ch, self.y.stride(0), n, len(self.so),
                                                 len(self.sh), self.stride, self.n_windows, _ptr(self.logits),
                                                 _ptr(self.ws), self.ws.numel(), _stream(stream)))

    def run(self):
        """Enqueue one scoring of every (segment, slide, window) on the plan's stream."""
        if self.graph is not None:
            self.graph.launch()
        else:
            self._enqueue(self.stream)
        return self.logits[:self.n_windows]
