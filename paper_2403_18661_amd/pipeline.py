"""The offline path as one object: Welch PSD -> whitening -> window scoring ->
integration, with every buffer allocated up front so that `run` only enqueues
library calls on one stream.

Geometry (paper Sec. VI): each hop of `psd_hop` whitened samples uses the PSD of
the `psd_len` raw samples that end `fduration/2` before the hop starts; the
first whitened sample therefore sits psd_len + fduration*fs/2 into the input.
With psd_len=None the PSD is taken over the whole input and only the filter
context (fduration/2 per edge) is cropped.
"""
from dataclasses import dataclass

import torch

from . import Net, integrate, lib, psd_estimate, whiten_apply, whiten_response, _workspace


@dataclass(frozen=True)
class PathConfig:
    fs: float = 2048.0
    prescale: float = 1e21
    nperseg: int = 4096
    noverlap: int = 2048
    psd_len: int = None          # samples of PSD background (None: whole input)
    psd_hop: int = 16384         # whitened samples per PSD (rolling background)
    fduration: float = 1.0       # whitening filter length in seconds
    highpass: float = 32.0
    stride: int = 128            # samples between windows (16 Hz)
    integrate_width: int = 16    # windows per 1 s at the stride above


class OfflinePath:
    def __init__(self, net: Net, n: int, cfg: PathConfig, device="cuda", batch=8192, x_dtype=torch.float64):
        self.net, self.cfg, self.n = net, cfg, n
        M = int(round(cfg.fduration * cfg.fs / 2))
        if cfg.psd_len is None:
            self.psd_len, self.n_psd, self.psd_hop = n, 1, 0
            self.out_start = M
            self.n_out = n - 2 * M
        else:
            self.psd_len = cfg.psd_len
            self.out_start = cfg.psd_len + M
            self.n_out = n - self.out_start - M
            self.psd_hop = cfg.psd_hop
            self.n_psd = -(-self.n_out // cfg.psd_hop)
        w = net.window
        self.n_windows = 0 if self.n_out < w else (self.n_out - w) // cfg.stride + 1
        n_ch = net.in_ch
        F = cfg.nperseg // 2 + 1
        L = lib()
        self.psd = torch.empty((self.n_psd, n_ch, F), dtype=torch.float64, device=device)
        self.ws_psd = _workspace(L.af_psd_workspace_bytes(n_ch, cfg.nperseg, cfg.noverlap, self.psd_len,
                                                          self.psd_hop, self.n_psd), device)
        self.y = torch.empty((n_ch, self.n_out), dtype=torch.float32, device=device)
        self.ws_wh = _workspace(L.af_whiten_workspace_bytes(n_ch, cfg.nperseg, self.n_psd), device)
        self.logits = torch.empty(self.n_windows, dtype=torch.float32, device=device)
        self.ws_net = _workspace(net.workspace_bytes(max(1, min(batch, self.n_windows))), device)
        self.integrated = torch.empty(max(self.n_windows - cfg.integrate_width + 1, 0), dtype=torch.float32,
                                      device=device)

    def psd_stage(self, x, stream=None):
        c = self.cfg
        return psd_estimate(x, c.fs, c.prescale, c.nperseg, c.noverlap, self.psd_len, self.psd_hop, self.n_psd,
                            out=self.psd, ws=self.ws_psd, stream=stream)

    def response_stage(self, stream=None):
        """Whitening filters of every PSD hop (af_whiten_response)."""
        c = self.cfg
        return whiten_response(self.psd, c.fs, c.fduration, c.highpass, out=self.ws_wh, stream=stream)

    def apply_stage(self, x, stream=None):
        """Overlap-save whitening with the hops' filters (af_whiten_apply)."""
        c = self.cfg
        return whiten_apply(x, self.ws_wh, self.n_psd, c.fs, c.prescale, self.psd_hop if self.n_psd > 1 else 0,
                            c.fduration, self.out_start, self.n_out, out=self.y, stream=stream)

    def whiten_stage(self, x, stream=None):
        self.response_stage(stream)
        return self.apply_stage(x, stream)

    def score_stage(self, stream=None):
        return self.net.score_windows(self.y, self.cfg.stride, self.n_windows, out=self.logits, ws=self.ws_net,
                                      stream=stream)

    def integrate_stage(self, stream=None):
        return integrate(self.logits, self.cfg.integrate_width, out=self.integrated, stream=stream)

    def run(self, x, stream=None):
        self.psd_stage(x, stream)
        self.whiten_stage(x, stream)
        self.score_stage(stream)
        self.integrate_stage(stream)
        return self.integrated
