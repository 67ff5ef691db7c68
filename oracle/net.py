"""1D residual scoring network, forward pass in FP64 (oracle).

The paper's detector maps a two-detector strain window to one scalar detection
statistic with a ResNet34-style network using 1D convolutions (Sec. II).  The
workloads here use folded BatchNorm and kernel 7; the forward pass is

    stem   : conv k, stride s0, 'same' zero padding -> BN -> ReLU [-> maxpool k3 s2 p1]
    block  : y = ReLU( BN2(conv2( ReLU(BN1(conv1(x))) )) + skip(x) ),
             skip = identity, or BN(conv 1x1 stride 2) when the shape changes
    head   : global average pool over time -> fully connected -> 1 logit

conv: out[c, t] = sum_{c', j} W[c, c', j] in[c', t*stride + j - (k-1)/2]
(zero outside the window), followed by eval-mode BN
    BN(v) = gamma (v - mean) / sqrt(var + eps) + beta,
which the fold turns into W' = W gamma / sqrt(var + eps), b' = beta - mean gamma / sqrt(var + eps).
The logit (not a sigmoid probability) is the detection statistic.

`net_forward_quant` emulates the low-precision GPU arithmetic exactly at every
rounding point (operands rounded to BF16 or scaled E4M3, products summed in
FP64, epilogue in the same order), to pin the BF16 and FP8 kernels more tightly
than the plain FP64 tolerance does.  For E4M3 it can also apply bias
correction: rounding the weights of a conv to E4M3 moves its output on average
by the weight error times the mean of its input, a systematic shift (the same
on every window) that dominates the FP8 logit error of the deep net; calibration
windows of noise give the input means, the shift is taken off each conv's bias,
and the mean logit shift that remains is taken off the FC bias.

Pins (tests/test_oracle_net.py): conv1d == brute-force loops and == torch's
float64 conv1d; folded == unfolded BatchNorm; the whole forward == a torch.nn
float64 model built from the same parameters; FLOP counts of both architectures.
The rounding points of net_forward_quant (tests/test_oracle_quant_points.py):
hand-worked logits of one-channel networks whose values sit on or between BF16
grid points, so that moving any rounding point changes a logit.
The E4M3 bias correction (tests/test_oracle_fp8_calib.py): hand-worked shifts of
a two-channel network; conv input means == forward hooks on the torch.nn model;
the FC shift centres the calibration logits; weights already on the grid need
no shift.
"""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

from .quant import bf16_round, e4m3_round, E4M3_MAX

BN_EPS = 1e-5


def fold_bn(w, gamma, beta, mean, var, eps=BN_EPS):
    s = gamma / np.sqrt(var + eps)
    return w * s[:, None, None], beta - mean * s


def conv1d(x, w, b, stride=1):
    """x [B, C_in, L], w [C_out, C_in, k] -> [B, C_out, L_out]; pad (k-1)/2."""
    k = w.shape[-1]
    pad = (k - 1) // 2
    B, C, L = x.shape
    L_out = (L + 2 * pad - k) // stride + 1
    xp = np.pad(x, ((0, 0), (0, 0), (pad, pad)))
    cols = sliding_window_view(xp, k, axis=2)[:, :, ::stride][:, :, :L_out]   # [B, C_in, L_out, k]
    out = np.tensordot(cols, w, axes=([1, 3], [1, 2]))                        # [B, L_out, C_out]
    return out.transpose(0, 2, 1) + b[None, :, None]


def maxpool3s2(x):
    """Max-pool, kernel 3, stride 2, padding 1 (padding never wins)."""
    B, C, L = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1)), constant_values=-np.inf)
    L_out = (L + 2 - 3) // 2 + 1
    return sliding_window_view(xp, 3, axis=2)[:, :, ::2][:, :, :L_out].max(axis=-1)


def folded_layers(params, arch):
    """Return dict name -> (W', b') for every conv, folding its BatchNorm."""
    out = {}

    def f(conv, bn):
        out[conv] = fold_bn(params[conv + ".w"], params[bn + ".gamma"], params[bn + ".beta"],
                            params[bn + ".mean"], params[bn + ".var"])

    f("stem.conv", "stem.bn")
    for pre, _, _, _, proj in arch.block_list():
        f(pre + ".conv1", pre + ".bn1")
        f(pre + ".conv2", pre + ".bn2")
        if proj:
            f(pre + ".proj", pre + ".projbn")
    return out


def net_forward(params, arch, x, return_features=False):
    """x [B, in_ch, window] float64 -> logits [B] (float64)."""
    L = folded_layers(params, arch)
    relu = lambda v: np.maximum(v, 0.0)
    h = relu(conv1d(x, *L["stem.conv"], stride=arch.stem_stride))
    if arch.stem_pool:
        h = maxpool3s2(h)
    for pre, _, _, stride, proj in arch.block_list():
        r = relu(conv1d(h, *L[pre + ".conv1"], stride=stride))
        r = conv1d(r, *L[pre + ".conv2"], stride=1)
        skip = conv1d(h, *L[pre + ".proj"], stride=stride) if proj else h
        h = relu(r + skip)
    g = h.mean(axis=2)
    logits = g @ params["fc.w"][0] + params["fc.b"][0]
    return (logits, g) if return_features else logits


def _f32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def _quant_conv(h, w, b, stride, precision):
    """One MFMA conv as the GPU computes it; h holds the stored (rounded) input."""
    if precision == "bf16":
        return conv1d(h, bf16_round(w), np.zeros_like(b), stride), None
    # fp8: per-window activation scale from the stored tensor's max |value|,
    # per-output-channel weight scale; the quantisation decisions are taken in
    # the same precision as the kernel (FP32 activation side, FP64 weight side)
    amax = np.abs(h).reshape(h.shape[0], -1).max(axis=1).astype(np.float32)
    amax = np.where(amax > 0, amax, np.float32(E4M3_MAX))
    inv = (np.float32(E4M3_MAX) / amax).astype(np.float32)
    s_a = (amax / np.float32(E4M3_MAX)).astype(np.float32)
    qa = e4m3_round((h.astype(np.float32) * inv[:, None, None]).astype(np.float32).astype(np.float64))
    s_w = np.abs(w).reshape(w.shape[0], -1).max(axis=1) / E4M3_MAX
    s_w = np.where(s_w > 0, s_w, 1.0)
    qw = e4m3_round(w / s_w[:, None, None])
    acc = conv1d(qa, qw, np.zeros_like(b), stride)
    deq = (s_a[:, None].astype(np.float32) * _f32(s_w)[None, :].astype(np.float32)).astype(np.float64)
    return acc, deq


def conv_input_means(params, arch, x):
    """Mean over windows and time of every MFMA conv's input, per input
    channel, in the FP64 network: dict conv name -> [C_in]."""
    L = folded_layers(params, arch)
    relu = lambda v: np.maximum(v, 0.0)
    mu = {}
    h = relu(conv1d(x, *L["stem.conv"], stride=arch.stem_stride))
    if arch.stem_pool:
        h = maxpool3s2(h)
    for pre, _, _, stride, proj in arch.block_list():
        mu[pre + ".conv1"] = h.mean(axis=(0, 2))
        r = relu(conv1d(h, *L[pre + ".conv1"], stride=stride))
        mu[pre + ".conv2"] = r.mean(axis=(0, 2))
        if proj:
            mu[pre + ".proj"] = h.mean(axis=(0, 2))
        skip = conv1d(h, *L[pre + ".proj"], stride=stride) if proj else h
        h = relu(conv1d(r, *L[pre + ".conv2"], stride=1) + skip)
    return mu


def fp8_weights(w):
    """Per-output-channel E4M3 weights, dequantised: s_c e4m3(W[c] / s_c),
    s_c = max|W[c]| / 448."""
    s_w = np.abs(w).reshape(w.shape[0], -1).max(axis=1) / E4M3_MAX
    s_w = np.where(s_w > 0, s_w, 1.0)
    return e4m3_round(w / s_w[:, None, None]) * s_w[:, None, None]


def fp8_bias_shift(params, arch, calib):
    """Bias correction of the E4M3 weights (reading R17): rounding a conv's
    weights moves its output, on average over representative inputs, by
    sum_{c', j} (W_q - W')[c, c', j] mu[c'], with mu the mean of the conv's
    input channels; that amount is taken off the conv's bias.  mu comes from
    the FP64 network on the calibration windows `calib` [B, in_ch, window].
    Returns dict conv name -> [C_out] shift (new bias = b' - shift)."""
    L = folded_layers(params, arch)
    mu = conv_input_means(params, arch, calib)
    return {name: np.einsum("ocj,c->o", fp8_weights(L[name][0]) - L[name][0], m) for name, m in mu.items()}


def _quant_core(L, arch, x, precision, fc_w, fc_b):
    relu = lambda v: np.maximum(v, 0.0)
    store = _f32 if precision == "bf16f" else bf16_round
    w0, b0 = L["stem.conv"]
    h = relu(conv1d(x, _f32(w0), _f32(b0), stride=arch.stem_stride))
    if arch.stem_pool:
        h = maxpool3s2(h)
    h = store(h)

    def run(hin, name, stride):
        w, b = L[name]
        if precision == "bf16f":
            acc, deq = _quant_conv(bf16_round(hin), w, b, stride, "bf16")
        else:
            acc, deq = _quant_conv(hin, w, b, stride, precision)
        bb = _f32(b)[None, :, None]
        return acc + bb if deq is None else acc * deq[:, :, None] + bb

    for pre, _, _, stride, proj in arch.block_list():
        r = store(relu(run(h, pre + ".conv1", stride)))
        skip = store(run(h, pre + ".proj", stride)) if proj else h
        h = store(relu(run(r, pre + ".conv2", 1) + skip))
    g = h.mean(axis=2)
    return g @ _f32(fc_w) + _f32(fc_b)[()]


def net_forward_quant(params, arch, x, precision, calib=None):
    """Emulate the GPU's low-precision network arithmetic; x [B, in_ch, window]
    holds float32-representable values.  Returns logits [B] (float64).

    'bf16f' (BF16 operands, FP32 activations): every stored tensor is rounded
    to FP32 and each conv rounds its input to BF16 as the operand; otherwise
    as 'bf16'.

    Stem: FP32 weights and input, vector arithmetic; its ReLU (and max-pool)
    output is stored as BF16.  Every other conv runs on the matrix cores with
    BF16 operands (precision 'bf16') or E4M3 operands with a per-window
    activation scale max|h|/448 and per-output-channel weight scales
    max|W'|/448 ('fp8'); the epilogue adds the FP32 bias (and, for the second
    conv of a block, the stored skip tensor), applies ReLU and stores BF16.
    Projections are stored as BF16 before the add.  GAP and FC run in FP32 on
    the stored BF16 activations.

    'fp8' with calibration windows `calib`: the network after bias correction
    (R17): every conv bias less fp8_bias_shift, and the FC bias less the mean
    difference, over the calibration windows, between the corrected FP8
    network's logits and the FP64 network's.
    """
    if precision not in ("bf16", "fp8", "bf16f"):
        raise ValueError(precision)
    L = folded_layers(params, arch)
    fc_w, fc_b = params["fc.w"][0], params["fc.b"][0]
    if calib is not None:
        if precision != "fp8":
            raise ValueError("calibration applies to the fp8 network")
        shift = fp8_bias_shift(params, arch, calib)
        L = {name: (w, b - shift[name]) if name in shift else (w, b) for name, (w, b) in L.items()}
        d_fc = np.mean(_quant_core(L, arch, calib, precision, fc_w, fc_b) - net_forward(params, arch, calib))
        fc_b = fc_b - d_fc
    return _quant_core(L, arch, x, precision, fc_w, fc_b)
