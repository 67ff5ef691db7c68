"""MI355X-native whitening + 1D-ResNet scoring for two-detector strain.

Thin Python binding over libaframe_mi.so (C ABI: include/aframe_mi.h).  Each
function marshals torch tensors (device memory) and the current HIP stream into
one C call; every step of the computation runs in the library's HIP kernels.
The functions follow the paper's pipeline (arXiv:2403.18661): Welch PSD of a
background stretch, whitening with an inverse-ASD FIR that loses 0.5 s per
edge, per-window scoring by a residual 1D CNN, 1 s top-hat integration.
"""
import ctypes

import numpy as np
import torch

from ._lib import AframeError, NetDesc, check, lib

__all__ = ["psd_estimate", "whiten", "Net", "integrate", "pack_params", "score_timeslides", "timeslide_n_windows",
           "AframeError", "lib"]

AF_IN_F64, AF_IN_F32 = 0, 1
PRECISIONS = {"f32": 0, "bf16": 1, "fp8": 2, "bf16f": 3}


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_dev(t, name, dtypes):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must have dtype in {dtypes}, got {t.dtype}")
    if t.numel() > 0 and t.stride(-1) != 1:
        raise ValueError(f"{name} must be contiguous in its last dimension")


def _in_dtype(x):
    return AF_IN_F64 if x.dtype == torch.float64 else AF_IN_F32


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def psd_estimate(x, fs, prescale=1.0, nperseg=4096, noverlap=None, psd_len=None, psd_hop=0, n_psd=1,
                 out=None, ws=None, stream=None):
    """Welch PSD of x [n_ch, n] -> [n_psd, n_ch, nperseg//2+1] float64 (af_psd_estimate)."""
    _check_dev(x, "x", (torch.float64, torch.float32))
    n_ch, n = x.shape
    noverlap = nperseg // 2 if noverlap is None else noverlap
    psd_len = n if psd_len is None else psd_len
    F = nperseg // 2 + 1
    if out is None:
        out = torch.empty((n_psd, n_ch, F), dtype=torch.float64, device=x.device)
    need = lib().af_psd_workspace_bytes(n_ch, nperseg, noverlap, psd_len, psd_hop, n_psd)
    ws = _workspace(need, x.device) if ws is None else ws
    check(lib().af_psd_estimate(_ptr(x), _in_dtype(x), n_ch, n, x.stride(0), fs, prescale, nperseg, noverlap,
                                psd_len, psd_hop, n_psd, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def whiten(x, psd, fs, prescale=1.0, psd_hop=0, fduration=1.0, highpass=32.0, out_start=None, n_out=None,
           out=None, ws=None, stream=None):
    """Whiten x [n_ch, n] with psd [n_psd, n_ch, F] -> y [n_ch, n_out] float32 (af_whiten).
    Default output range: crop fduration/2 at each edge."""
    _check_dev(x, "x", (torch.float64, torch.float32))
    _check_dev(psd, "psd", (torch.float64,))
    if psd.dim() == 2:
        psd = psd.unsqueeze(0)
    n_psd, _, F = psd.shape
    nperseg = 2 * (F - 1)
    n_ch, n = x.shape
    M = int(round(fduration * fs / 2))
    out_start = M if out_start is None else out_start
    n_out = n - out_start - M if n_out is None else n_out
    if out is None:
        out = torch.empty((n_ch, n_out), dtype=torch.float32, device=x.device)
    need = lib().af_whiten_workspace_bytes(n_ch, nperseg, n_psd)
    ws = _workspace(need, x.device) if ws is None else ws
    check(lib().af_whiten(_ptr(x), _in_dtype(x), n_ch, n, x.stride(0), fs, prescale, _ptr(psd.contiguous()),
                          nperseg, n_psd, psd_hop, fduration, highpass, out_start, n_out, _ptr(out),
                          out.stride(0), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def whiten_response(psd, fs, fduration=1.0, highpass=32.0, out=None, stream=None):
    """Whitening filters of psd [n_psd, n_ch, F] into a device buffer
    (af_whiten_response); pass it to whiten_apply."""
    _check_dev(psd, "psd", (torch.float64,))
    if psd.dim() == 2:
        psd = psd.unsqueeze(0)
    n_psd, n_ch, F = psd.shape
    nperseg = 2 * (F - 1)
    need = lib().af_whiten_workspace_bytes(n_ch, nperseg, n_psd)
    out = _workspace(need, psd.device) if out is None else out
    check(lib().af_whiten_response(_ptr(psd.contiguous()), n_ch, nperseg, n_psd, fs, fduration, highpass, _ptr(out),
                                   out.numel(), _stream(stream)))
    return out


def whiten_apply(x, resp, n_psd, fs, prescale=1.0, psd_hop=0, fduration=1.0, out_start=None, n_out=None, out=None,
                 stream=None):
    """Whiten x [n_ch, n] with filters from whiten_response (af_whiten_apply)."""
    _check_dev(x, "x", (torch.float64, torch.float32))
    n_ch, n = x.shape
    M = int(round(fduration * fs / 2))
    out_start = M if out_start is None else out_start
    n_out = n - out_start - M if n_out is None else n_out
    if out is None:
        out = torch.empty((n_ch, n_out), dtype=torch.float32, device=x.device)
    check(lib().af_whiten_apply(_ptr(x), _in_dtype(x), n_ch, n, x.stride(0), fs, prescale, _ptr(resp), resp.numel(),
                                n_psd, psd_hop, fduration, out_start, n_out, _ptr(out), out.stride(0),
                                _stream(stream)))
    return out


def pack_params(params, arch):
    """Flatten a name -> array parameter dict into the C ABI's order: per conv
    (stem; per block conv1, conv2, [proj]) weight then BN gamma, beta, mean,
    var (GroupNorm nets: gamma, beta); then FC weight and bias.  `arch`
    provides block_list() and norm."""
    parts = []

    keys = ("gamma", "beta") if getattr(arch, "norm", "bn") == "gn" else ("gamma", "beta", "mean", "var")

    def conv(c, bn):
        parts.append(np.asarray(params[c + ".w"], np.float64).ravel())
        for k in keys:
            parts.append(np.asarray(params[f"{bn}.{k}"], np.float64).ravel())

    conv("stem.conv", "stem.bn")
    for pre, _, _, _, proj in arch.block_list():
        conv(pre + ".conv1", pre + ".bn1")
        conv(pre + ".conv2", pre + ".bn2")
        if proj:
            conv(pre + ".proj", pre + ".projbn")
    parts.append(np.asarray(params["fc.w"], np.float64).ravel())
    parts.append(np.asarray(params["fc.b"], np.float64).ravel())
    return np.ascontiguousarray(np.concatenate(parts))


class Net:
    """A scoring network resident on the current device (af_net_create; for an
    architecture with norm "gn", af_net_create_gn)."""

    def __init__(self, arch, params, precision="f32"):
        d = NetDesc()
        d.in_ch, d.stem_ch, d.kernel = arch.in_ch, arch.stem_ch, arch.kernel
        d.stem_stride, d.stem_pool, d.n_stages = arch.stem_stride, int(arch.stem_pool), len(arch.widths)
        for i, (w, b) in enumerate(zip(arch.widths, arch.blocks)):
            d.widths[i], d.blocks[i] = w, b
        d.window = arch.window
        flat = params if isinstance(params, np.ndarray) else pack_params(params, arch)
        flat = np.ascontiguousarray(flat, dtype=np.float64)
        self.window = arch.window
        self.in_ch = arch.in_ch
        self.precision = precision
        self.norm = getattr(arch, "norm", "bn")
        h = ctypes.c_void_p()
        if getattr(arch, "norm", "bn") == "gn":
            check(lib().af_net_create_gn(ctypes.byref(d), arch.groups, flat.ctypes.data_as(ctypes.c_void_p),
                                         flat.size, PRECISIONS[precision], ctypes.byref(h)))
        else:
            check(lib().af_net_create(ctypes.byref(d), flat.ctypes.data_as(ctypes.c_void_p), flat.size,
                                      PRECISIONS[precision], ctypes.byref(h)))
        self._h = h

    def close(self):
        """Free the device weights now (also done when the object is collected)."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().af_net_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: the library may already be unloaded
            pass

    @property
    def macs(self):
        return lib().af_net_macs(self._h)

    @property
    def fused(self):
        """True when scoring runs as the whole-network persistent kernel."""
        return bool(lib().af_net_fused(self._h))

    @fused.setter
    def fused(self, enable):
        check(lib().af_net_set_fused(self._h, int(bool(enable))))

    def fused_tile(self):
        """(rows per step, candidates, chosen) of the whole-network kernel."""
        v = [ctypes.c_int32() for _ in range(3)]
        check(lib().af_net_fused_tile(self._h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_fused_tile(self, chosen):
        check(lib().af_net_set_fused_tile(self._h, chosen))

    @property
    def n_layers(self):
        return lib().af_net_n_layers(self._h)

    @property
    def n_convs(self):
        """MFMA conv layers (profile layers 1 .. n_convs)."""
        return self.n_layers - (3 if self.norm == "gn" else 2)

    def profile_begin(self):
        """Start per-kernel HIP-event timing of score_windows calls."""
        check(lib().af_net_profile_begin(self._h))

    def profile_end(self):
        """Stop timing; return per-layer dict arrays ms, launches, flops
        (layer 0 = stem, then convs in execution order, then the head; GroupNorm
        nets end with one more entry, the separate GroupNorm launches)."""
        n = self.n_layers
        ms = np.zeros(n)
        la = np.zeros(n, dtype=np.int64)
        fl = np.zeros(n)
        check(lib().af_net_profile_end(self._h, n, ms.ctypes.data_as(ctypes.c_void_p),
                                       la.ctypes.data_as(ctypes.c_void_p), fl.ctypes.data_as(ctypes.c_void_p)))
        return {"ms": ms, "launches": la, "flops": fl}

    def autotune(self, batch=1024, ws=None, stream=None):
        """Time every candidate tile shape per conv layer and keep the fastest
        (af_net_autotune); returns the number of layers that changed."""
        if ws is None:
            ws = _workspace(self.workspace_bytes(batch), "cuda")
        n = ctypes.c_int64()
        check(lib().af_net_autotune(self._h, batch, _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(n)))
        return n.value

    def tiles(self):
        """[(rows, out_channels, n_candidates, chosen)] per conv layer."""
        out = []
        for layer in range(1, self.n_convs + 1):
            v = [ctypes.c_int32() for _ in range(4)]
            check(lib().af_net_layer_tile(self._h, layer, *[ctypes.byref(x) for x in v]))
            out.append(tuple(x.value for x in v))
        return out

    def set_tile(self, layer, chosen):
        """Use tile candidate `chosen` for conv layer `layer` (1 = first conv;
        af_net_set_layer_tile)."""
        check(lib().af_net_set_layer_tile(self._h, layer, chosen))

    def workspace_bytes(self, batch):
        return lib().af_score_workspace_bytes(self._h, batch)

    def calibrate(self, y, stride, n_windows=None, batch=256, stream=None):
        """Bias correction of an FP8 net from the windows of y [n_ch, n]
        float32 (af_net_calibrate; synchronous)."""
        _check_dev(y, "y", (torch.float32,))
        n_ch, n = y.shape
        if n_windows is None:
            n_windows = (n - self.window) // stride + 1
        ws = _workspace(2 * self.workspace_bytes(max(1, min(batch, n_windows))), y.device)
        check(lib().af_net_calibrate(self._h, _ptr(y), n_ch, y.stride(0), n, stride, n_windows, _ptr(ws),
                                     ws.numel(), _stream(stream)))

    def score_windows(self, y, stride, n_windows=None, shifts=None, wrap=0, batch=1024, out=None, ws=None,
                      stream=None):
        """Logits of windows of y [n_ch, n] float32 (af_score_windows)."""
        _check_dev(y, "y", (torch.float32,))
        n_ch, n = y.shape
        if n_windows is None:
            n_windows = 0 if n < self.window else (n - self.window) // stride + 1
        if out is None:
            out = torch.empty(n_windows, dtype=torch.float32, device=y.device)
        if ws is None:
            ws = _workspace(self.workspace_bytes(max(1, min(batch, n_windows))), y.device)
        sh = None
        if shifts is not None:
            sh = (ctypes.c_int64 * n_ch)(*[int(v) for v in shifts])
        check(lib().af_score_windows(self._h, _ptr(y), n_ch, y.stride(0), n, stride, n_windows,
                                     ctypes.cast(sh, ctypes.c_void_p) if sh is not None else None, wrap,
                                     _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
        return out


def _i64(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.int64))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def timeslide_n_windows(seg_len, n_slides, window=3072, stride=2048):
    a, p = _i64(seg_len)
    return int(lib().af_timeslide_n_windows(p, len(a), n_slides, window, stride))


def score_timeslides(net, y, seg_off, seg_len, shifts, stride=2048, batch=4096, out=None, ws=None, stream=None):
    """Logits of every (segment, slide, window) of a timeslide background
    (af_score_timeslides); y [n_ch, n] float32 holds the whitened segments."""
    _check_dev(y, "y", (torch.float32,))
    n_ch, n = y.shape
    so, pso = _i64(seg_off)
    sl, psl = _i64(seg_len)
    sh, psh = _i64(shifts)
    tot = timeslide_n_windows(sl, len(sh), net.window, stride)
    if out is None:
        out = torch.empty(tot, dtype=torch.float32, device=y.device)
    if ws is None:
        ws = _workspace(lib().af_timeslide_workspace_bytes(net._h, len(so), len(sh), max(1, min(batch, tot))),
                        y.device)
    check(lib().af_score_timeslides(net._h, _ptr(y), n_ch, y.stride(0), n, pso, psl, len(so), psh, len(sh), stride,
                                    _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def integrate(p, width, carry=None, out=None, stream=None):
    """Causal 1 s top-hat mean of logits p [n] (af_integrate): -> [n - width + 1]
    in valid mode, or, with carry (float32 [width - 1] device tensor holding the
    predictions that precede p, updated in place), -> [n], one per new
    prediction."""
    _check_dev(p, "p", (torch.float32,))
    n = p.numel()
    if carry is not None:
        _check_dev(carry, "carry", (torch.float32,))
        if carry.numel() != width - 1:
            raise ValueError(f"carry must hold width - 1 = {width - 1} values")
    m = n if carry is not None else max(n - width + 1, 0)
    if out is None:
        out = torch.empty(m, dtype=torch.float32, device=p.device)
    check(lib().af_integrate(_ptr(p), n, width, _ptr(carry) if carry is not None and carry.numel() else None,
                             _ptr(out), _stream(stream)))
    return out


def cluster(x, half, offsets=None, max_out=None, stream=None):
    """Candidate events of the statistic x [n] (af_cluster): sample i is kept
    iff it beats every sample up to `half` before it and ties or beats every
    sample up to `half` after it, within its series (offsets: int64 [n_series
    + 1] device tensor, or None for one series).  Returns (idx int64, val
    float32) device tensors, ascending; waits for the count."""
    _check_dev(x, "x", (torch.float32,))
    n = x.numel()
    n_series = 1
    if offsets is not None:
        _check_dev(offsets, "offsets", (torch.int64,))
        n_series = offsets.numel() - 1
    if max_out is None:
        max_out = n
    idx = torch.empty(max(max_out, 1), dtype=torch.int64, device=x.device)
    val = torch.empty(max(max_out, 1), dtype=torch.float32, device=x.device)
    found = torch.empty(1, dtype=torch.int64, device=x.device)
    ws = _workspace(lib().af_cluster_workspace_bytes(n), x.device)
    check(lib().af_cluster(_ptr(x), n, _ptr(offsets) if offsets is not None else None, n_series, half, _ptr(idx),
                           _ptr(val), max_out, _ptr(found), _ptr(ws), ws.numel(), _stream(stream)))
    k = min(int(found.item()), max_out)
    return idx[:k], val[:k]


def project(hp, hc, sky, det, fs=2048.0, out=None, stream=None):
    """Polarisations hp, hc [n_inj, len] float32 projected onto detectors
    (af_project); sky [n_inj, 4] float64 device (ra, dec, psi, gmst); det:
    host array [n_det, 9] (vertex m, x arm, y arm).  -> [n_inj, n_det, len]."""
    _check_dev(hp, "hp", (torch.float32,))
    _check_dev(hc, "hc", (torch.float32,))
    _check_dev(sky, "sky", (torch.float64,))
    det = np.ascontiguousarray(det, dtype=np.float64).reshape(-1, 9)
    n_inj, n = hp.shape
    if out is None:
        out = torch.empty((n_inj, det.shape[0], n), dtype=torch.float32, device=hp.device)
    check(lib().af_project(_ptr(hp), _ptr(hc), n_inj, n, float(fs), det.ctypes.data_as(ctypes.c_void_p),
                           det.shape[0], _ptr(sky), _ptr(out), _stream(stream)))
    return out


def snr_rescale(sig, psd, df, fs=2048.0, f_low=20.0, target=None, stream=None):
    """Network optimal SNR of sig [n_inj, n_det, len] against psd [n_det,
    n_freq] float64 on the grid m*df (af_snr_rescale); with target
    [n_inj] float64, sig is scaled in place to it.  Returns snr float64."""
    _check_dev(sig, "sig", (torch.float32,))
    _check_dev(psd, "psd", (torch.float64,))
    n_inj, n_det, n = sig.shape
    snr = torch.empty(n_inj, dtype=torch.float64, device=sig.device)
    if target is not None:
        _check_dev(target, "target", (torch.float64,))
    check(lib().af_snr_rescale(_ptr(sig), n_inj, n_det, n, float(fs), _ptr(psd), psd.shape[-1], float(df),
                               float(f_low), _ptr(target) if target is not None else None, _ptr(snr),
                               _stream(stream)))
    return snr


def far(bg, livetime, x, stream=None):
    """False alarm rates (af_far): #{background > x[q]} / livetime per query,
    FP64 [n_q]."""
    _check_dev(bg, "bg", (torch.float32,))
    _check_dev(x, "x", (torch.float32,))
    out = torch.empty(x.numel(), dtype=torch.float64, device=x.device)
    ws = _workspace(lib().af_far_workspace_bytes(x.numel()), x.device)
    check(lib().af_far(_ptr(bg) if bg.numel() else None, bg.numel(), float(livetime), _ptr(x), x.numel(), _ptr(out),
                       _ptr(ws), ws.numel(), _stream(stream)))
    return out
