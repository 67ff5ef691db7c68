/*
 * aframe_mi.h — C ABI of the MI355X (gfx950) whitening + 1D-ResNet scoring library.
 *
 * The library implements the data-parallel hot path of a machine-learning
 * search for compact-binary-coalescence gravitational waves (Aframe,
 * arXiv:2403.18661): estimate each detector's noise PSD (Sec. IV.B noise
 * sampling, Sec. VI), build an inverse-ASD whitening filter and whiten the
 * strain, cropping the filter's 0.5 s settle-in at each edge (Sec. IV.B,
 * Table III), score overlapping 1.5 s two-detector windows with a 1D residual
 * CNN that returns one scalar detection statistic per window (Sec. II), and
 * smooth the statistic with a 1 s top hat (Sec. II).
 *
 * Conventions shared by every entry point
 *  - All data pointers are DEVICE pointers on the current HIP device unless a
 *    parameter says "host".  The caller owns every buffer (inputs, outputs and
 *    workspace); the library owns only af_net, af_graph and af_server objects
 *    and its constant tables (FFT twiddles), which sit in static device arrays
 *    of the library's code object (nothing is allocated for them).
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = default stream).
 *    The constant tables are computed by a kernel that the first call needing
 *    them on a device queues on its own stream (calls on other streams wait
 *    for it on the device, not on the host), or eagerly by af_init.  Calls
 *    that synchronise say so: af_init, af_net_create(_gn), af_net_calibrate,
 *    af_net_autotune, af_net_set_layer_tile, af_timeslide_prepare (and
 *    af_score_timeslides through it) and the streaming server's calls.
 *  - Every argument is validated on the host before anything is launched; an
 *    invalid call returns AF_EINVAL and leaves outputs untouched.  HIP runtime
 *    failures return AF_EHIP.  af_last_error() returns a message for the last
 *    failing call on the calling thread.
 *  - Calls on distinct streams and distinct workspaces may run concurrently;
 *    one af_net may be used from several streams at once (it is read-only).
 */
#ifndef AFRAME_MI_H
#define AFRAME_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AF_OK = 0,
    AF_EINVAL = -1,        /* bad argument or shape; nothing launched            */
    AF_ENOMEM = -2,        /* host or device allocation failed                  */
    AF_EHIP = -3,          /* HIP runtime error (message in af_last_error)      */
    AF_EUNSUPPORTED = -4,  /* valid request that this build does not implement  */
    AF_EBUDGET = -5        /* the HBM budget (or stream slots) would be exceeded */
} af_status;

typedef void* af_stream;   /* hipStream_t */

typedef enum { AF_IN_F64 = 0, AF_IN_F32 = 1 } af_dtype;
/* Conv arithmetic.  AF_F32: FP32 operands and activations.  AF_BF16: BF16
 * operands and BF16 stored activations.  AF_FP8: E4M3 operands (per-channel
 * weight scales, per-window activation scales), BF16 stored activations.
 * AF_BF16_F32ACT: BF16 operands, FP32 stored activations (the residual
 * stream keeps FP32; operands are rounded to BF16 as they are loaded).  The
 * inner activation of a residual block, read only as the operand of the
 * block's second conv, is stored already rounded to BF16, which gives the
 * same result with half its traffic.  All accumulate in FP32; the stem conv
 * is FP32 in every mode. */
typedef enum { AF_F32 = 0, AF_BF16 = 1, AF_FP8 = 2, AF_BF16_F32ACT = 3 } af_precision;

/* Message describing the last error on this thread ("" if none). */
const char* af_last_error(void);
/* Builds the current device's constant tables now and waits for them.
 * Optional: without it the first call that needs them builds them on its
 * stream.  Call it once per device before capturing a graph of the PSD,
 * whitening or SNR entry points (their first call cannot queue the build into
 * a capture and returns AF_EINVAL instead). */
af_status af_init(void);
/* Library version string. */
const char* af_version(void);

/* ------------------------------------------------------------------------
 * Welch PSD (Sec. IV.B noise sampling; Sec. VI: "the first 64 seconds ... to
 * estimate the PSD").  One-sided PSD with periodic-Hann segments of `nperseg`
 * samples every nperseg - noverlap samples, mean of |rFFT|^2 over segments,
 * density scaling c_k / (fs sum w^2) with c_0 = c_{nperseg/2} = 1, else 2.
 *
 * x      : [n_ch][ld_x] strain (AF_IN_F64: physical strain, AF_IN_F32: any
 *          float series); every sample is multiplied by `prescale` on load
 *          (1e21 brings physical strain to O(1)).
 * PSD j (j < n_psd) is estimated from x[:, j*psd_hop : j*psd_hop + psd_len]
 * (a rolling background); psd_hop must be a multiple of nperseg - noverlap
 * when n_psd > 1.  With n_psd = 1, psd_hop is ignored.
 * psd    : [n_psd][n_ch][nperseg/2 + 1] float64 output, in (prescale*x)^2/Hz.
 * nperseg: power of two in [256, 4096].
 * Segment spectra and averaging are computed in FP64.
 * ws     : device workspace of at least af_psd_workspace_bytes(...) bytes.
 * ------------------------------------------------------------------------ */
size_t af_psd_workspace_bytes(int64_t n_ch, int64_t nperseg, int64_t noverlap,
                              int64_t psd_len, int64_t psd_hop, int64_t n_psd);
af_status af_psd_estimate(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x,
                          double fs, double prescale, int64_t nperseg, int64_t noverlap,
                          int64_t psd_len, int64_t psd_hop, int64_t n_psd,
                          double* psd, void* ws, size_t ws_bytes, af_stream stream);

/* ------------------------------------------------------------------------
 * Whitening (Sec. IV.B: PSD -> whitening filter -> whiten in the frequency
 * domain -> crop 0.5 s per edge; Sec. VI; Table III, the row for cropping
 * the filter's corrupted edges).  The filter is the inverse ASD with bins below
 * `highpass` zeroed, transformed to a zero-phase impulse response and
 * truncated with a Hann taper to |m| < M = fduration*fs/2 taps per side:
 *     y[c][i] = sqrt(2/fs) * sum_m h_j[c][m] * prescale * x[c][out_start + i - m]
 * for i < n_out, with j = min(i / psd_hop, n_psd - 1).  In-band white output
 * has unit variance.  The filter is built in FP64 on the device; the
 * convolution runs as FP32 overlap-save FFTs of 8192 points.
 *
 * psd    : [n_psd][n_ch][nperseg/2+1] float64 (as written by af_psd_estimate
 *          with the same prescale).  nperseg in {2048, 4096}, 2M-1 <= nperseg.
 * Context: out_start >= M and out_start + n_out + M <= n.
 * y      : [n_ch][ld_y] float32 output, ld_y >= n_out.
 * ------------------------------------------------------------------------ */
size_t af_whiten_workspace_bytes(int64_t n_ch, int64_t nperseg, int64_t n_psd);
af_status af_whiten(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x,
                    double fs, double prescale, const double* psd, int64_t nperseg,
                    int64_t n_psd, int64_t psd_hop, double fduration, double highpass,
                    int64_t out_start, int64_t n_out, float* y, int64_t ld_y,
                    void* ws, size_t ws_bytes, af_stream stream);

/* af_whiten without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments minus ws and ws_bytes, the same kernels and
 * the same output bit for bit.  The filter responses go to a static scratch
 * array of 16 MiB + 4 KiB per GPU (512 (PSD, detector pair) combinations of
 * af_whiten_workspace_bytes, e.g. 512 PSDs of one or two detectors, 256 of
 * three or four), held from when the library's code loads on the GPU until
 * the process ends; larger requests return AF_EINVAL.  It calls no allocation
 * routine (af_init looks up the array's address; otherwise the first call on
 * a device does).  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (several streams or threads) race and must be
 * serialised by the caller. */
af_status af_whiten_noalloc(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double fs,
                            double prescale, const double* psd, int64_t nperseg, int64_t n_psd, int64_t psd_hop,
                            double fduration, double highpass, int64_t out_start, int64_t n_out, float* y,
                            int64_t ld_y, af_stream stream);

/* The two halves of af_whiten, for callers that reuse filters (one rolling
 * PSD serving several output spans) or time them apart.
 * af_whiten_response builds the filters of n_psd PSDs (FP64 on the device,
 * stored as float) into resp: device memory of at least
 * af_whiten_workspace_bytes(n_ch, nperseg, n_psd) bytes, caller-owned, whose
 * layout is private to the library.
 * af_whiten_apply convolves x with filters made by af_whiten_response for the
 * same n_ch, fs and fduration; x, n, ld_x, prescale, n_psd, psd_hop,
 * out_start, n_out, y and ld_y mean what they mean for af_whiten and are
 * checked the same way.  Both return AF_EINVAL before any launch on a bad
 * argument or a buffer that is too small; af_whiten_apply also rejects a resp
 * that no af_whiten_response call of this process filled, or one filled for
 * another filter length (fduration*fs/2), another channel count or fewer
 * PSDs (the library records what each af_whiten_response call built, by
 * buffer address). */
af_status af_whiten_response(const double* psd, int64_t n_ch, int64_t nperseg, int64_t n_psd, double fs,
                             double fduration, double highpass, void* resp, size_t resp_bytes,
                             af_stream stream);
af_status af_whiten_apply(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double fs,
                          double prescale, const void* resp, size_t resp_bytes, int64_t n_psd,
                          int64_t psd_hop, double fduration, int64_t out_start, int64_t n_out, float* y,
                          int64_t ld_y, af_stream stream);

/* ------------------------------------------------------------------------
 * Scoring network (Sec. II: 1D-convolutional ResNet mapping a two-detector
 * window to one scalar detection statistic).  Architecture: stem conv (kernel
 * k, stride stem_stride) + BN + ReLU [+ max-pool 3/2/1]; n_stages stages of
 * BasicBlocks (conv-BN-ReLU-conv-BN + skip, ReLU), stride 2 at the first block
 * of stages > 0, 1x1 conv + BN projection where the shape changes; global
 * average pool; FC -> 1 logit.  BatchNorm is folded into the convs
 * (eval mode, eps 1e-5) when the net is created.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t in_ch;        /* detectors (2)                       */
    int32_t stem_ch;      /* stem output channels                */
    int32_t kernel;       /* conv kernel size (odd)              */
    int32_t stem_stride;  /* 1 or 2                              */
    int32_t stem_pool;    /* 1: max-pool k3 s2 p1 after the stem */
    int32_t n_stages;     /* <= 8                                */
    int32_t widths[8];
    int32_t blocks[8];
    int32_t window;       /* samples per window (3072 = 1.5 s)   */
} af_net_desc;

typedef struct af_net af_net;

/* params (host, float64): for each conv in execution order (stem; then per
 * block conv1, conv2, [proj]) its weight [C_out][C_in][k] followed by its BN
 * gamma, beta, running_mean, running_var [C_out]; then fc weight [C_last] and
 * fc bias [1].  n_params must equal the total.  Weights are folded in FP64 and
 * stored in `precision` (FP8: E4M3 with per-output-channel scales max|W'|/448).
 * Synchronous.  *out receives the handle. */
af_status af_net_create(const af_net_desc* desc, const double* params, int64_t n_params,
                        af_precision precision, af_net** out);
/* The paper's own form of the network (Sec. II: GroupNorm in place of
 * BatchNorm; Sec. IX: convolutions of kernel length 3 with global pooling):
 * every conv has no bias and is followed by GroupNorm with `groups` groups of
 * consecutive channels (per window: mean and biased variance over the group's
 * channels and all samples, eps 1e-5, then per-channel gamma, beta), in the
 * same places as the BatchNorms of af_net_create's network (stem, each conv of
 * a block, each projection).  params (host, float64): per conv, weight
 * [C_out][C_in][k] then gamma [C_out], beta [C_out]; then fc weight [C_last]
 * and fc bias [1].  desc->kernel must be 3; stem_ch a power of two in
 * [16, 256] and every width a power of two in [16, 1024], each divisible by
 * groups (the standard ResNet34 widths 64/128/256/512 included); precision
 * AF_F32, or AF_BF16_F32ACT
 * (BF16 conv operands, FP32 activations and GroupNorm); in_ch must be 2.
 * The handle works with af_score_windows, the timeslide entry points, the
 * streaming server, the autotuner and the profile; statistics are taken per
 * window, so a window's logit does not depend on its batch.  AF_EINVAL on a
 * bad shape or length. */
af_status af_net_create_gn(const af_net_desc* desc, int32_t groups, const double* params, int64_t n_params,
                           af_precision precision, af_net** out);
/* Bias correction of an AF_FP8 net from calibration windows (E4M3 weight
 * rounding moves each conv's output by the same amount on every window: the
 * weight error times the mean of the conv's input; that systematic shift, not
 * the per-window rounding noise, is most of the FP8 logit error of a deep
 * net).  The windows of y (as for af_score_windows without shifts: window i
 * starts at i*stride; noise of the statistics the net will see, e.g. whitened
 * noise) are scored by the same network in FP32, whose activations give mu,
 * the mean of every conv input per channel over windows and time.  Each conv
 * bias b' becomes b' - sum_{c,j} (s e4m3(W'/s) - W')[o][c][j] mu[c] (FP64 on
 * the host, from the weights as created), then the FC bias is lowered by the
 * mean, over the calibration windows, of (FP8 logit - FP32 logit) with the
 * corrected convs.  The result depends only on the calibration windows
 * (calling again recomputes from the created weights).  Synchronous: it
 * waits for the device, allocates its own scratch and replaces the biases in
 * place, so graphs captured with this net replay with the new biases; work
 * queued with the net on other streams must be complete.  ws must hold at
 * least af_score_workspace_bytes() of the FP32 form for one window (twice
 * that of the FP8 net); windows run in passes of what it holds.  AF_EINVAL
 * for a net that is not FP8 (GroupNorm nets included) or windows past n. */
af_status af_net_calibrate(af_net* net, const float* y, int64_t n_ch, int64_t ld_y, int64_t n, int64_t stride,
                           int64_t n_windows, void* ws, size_t ws_bytes, af_stream stream);
void af_net_destroy(af_net* net);
/* Total conv + FC multiply-accumulates per window. */
int64_t af_net_macs(const af_net* net);

/* Whole-network path.  For the 16-channel two-block net (stem 2->16 k7 s1,
 * one stage of two BasicBlocks) in BF16, scoring runs as one persistent kernel
 * (one wavefront per window, every activation in LDS; on by default).
 * af_net_fused reports whether it is active; af_net_set_fused(net, 0) selects
 * the layer-by-layer kernels instead (AF_EINVAL if enabling it on a net
 * without the path).  The kernel walks a window in steps of `rows` time rows;
 * af_net_fused_tile reports the candidates' count and the one in use, which
 * af_net_autotune picks by timing and af_net_set_fused_tile sets (logits are
 * the same bit for bit under every candidate). */
int af_net_fused(const af_net* net);
af_status af_net_set_fused(af_net* net, int enable);
af_status af_net_fused_tile(const af_net* net, int32_t* rows, int32_t* n_candidates, int32_t* chosen);
af_status af_net_set_fused_tile(af_net* net, int32_t chosen);

/* Number of timed layers: stem, each conv in execution order, GAP+FC head;
 * GroupNorm nets (af_net_create_gn) have one more, after the head, that
 * collects the blocks' separate GroupNorm launches (scale and shift of every
 * conv's norm, each block's end); the stem's norm runs inside the stem kernel
 * (layer 0). */
int64_t af_net_n_layers(const af_net* net);
/* Kernel timing (a tracing aid, Sec. VIII reports per-stage latencies).
 * Between begin and end, every af_score_windows call on this net records a HIP
 * event pair around each kernel it launches (on the call's stream).  end()
 * waits for those events and writes, per layer index (0 = stem, 1.. = convs
 * in execution order, last = head): total milliseconds, launch count and
 * algorithmic FLOPs (2 x MACs x windows).  With the whole-network kernel the
 * entire network's time and FLOPs are reported under layer 1.  Arrays have af_net_n_layers()
 * entries.  Not thread-safe with concurrent scoring on the same net. */
af_status af_net_profile_begin(af_net* net);
af_status af_net_profile_end(af_net* net, int64_t n_layers, double* ms, int64_t* launches, double* flops);

/* Conv tile autotuner.  Every conv layer has a few candidate tile shapes
 * (rows x output channels per workgroup, LDS buffering); this times each one
 * on `batch` windows (contents of ws are overwritten; ws must hold
 * af_score_workspace_bytes(net, batch)) and keeps the fastest, rebuilding that
 * layer's weight image.  The whole-network kernel's candidates are timed in
 * its steady state instead: on 256 windows per CU (fewer if ws holds fewer)
 * of ws read as a two-channel series.  Synchronous; results are unchanged up to the
 * tile-independent per-window arithmetic (the same logits bit for bit).
 * *n_changed (may be NULL) receives the number of layers switched. */
af_status af_net_autotune(af_net* net, int64_t batch, void* ws, size_t ws_bytes, af_stream stream,
                          int64_t* n_changed);
/* Tile in use for conv layer `layer` (1 = first conv, as in the profile):
 * rows (mt) and output channels (nt) per workgroup, candidate count, chosen index. */
af_status af_net_layer_tile(const af_net* net, int64_t layer, int32_t* mt, int32_t* nt, int32_t* n_candidates,
                            int32_t* chosen);
/* Use tile candidate `chosen` (0 <= chosen < n_candidates) for conv layer
 * `layer`, e.g. to replay an earlier autotuning without timing again.  Waits
 * for the device, then rebuilds the layer's weight image; logits are the same
 * bit for bit under every candidate.  AF_EINVAL for a bad layer or index.
 * A replaced weight image (here or in af_net_autotune) stays allocated until
 * af_net_destroy, so a graph captured before the switch still replays with
 * the old tile and image, giving the same logits. */
af_status af_net_set_layer_tile(af_net* net, int64_t layer, int32_t chosen);

/* Workspace needed to score `batch` windows per internal pass. */
size_t af_score_workspace_bytes(const af_net* net, int64_t batch);
/* logits[i] = net(window i) for i < n_windows.  Channel c of window i is
 *   y[c*ld_y + p], p = i*stride + ch_shift[c] + t, t < window,
 * with p taken modulo `wrap` when wrap > 0 (circular timeslides, Sec. IX);
 * wrap must then be at least the window length (AF_EINVAL otherwise).
 * ch_shift: host array [n_ch] or NULL (all 0).  Without wrap every p must be
 * < n.  y is float32; it is rounded to the net's precision inside the kernels.
 * Windows are processed in passes of the largest batch the workspace holds. */
af_status af_score_windows(const af_net* net, const float* y, int64_t n_ch, int64_t ld_y,
                           int64_t n, int64_t stride, int64_t n_windows,
                           const int64_t* ch_shift, int64_t wrap, float* logits,
                           void* ws, size_t ws_bytes, af_stream stream);

/* ------------------------------------------------------------------------
 * Timeslide background (Sec. IX: H1 held fixed, L1 shifted in 1 s steps to
 * build background livetime).  Segment s occupies samples
 * [seg_off[s], seg_off[s] + seg_len[s]) of every channel of y (host arrays).
 * For slide k and window i of segment s, channel 0 reads samples
 * i*stride + t and every other channel reads (i*stride + shifts[k] + t) mod
 * seg_len[s], t < window, both relative to seg_off[s] (circular shift inside
 * the segment).  A segment holds (seg_len - window)/stride + 1 windows (none if
 * shorter than a window).  logits are written segment-major, then slide, then
 * window: [sum_s n_slides * n_w(s)] floats, af_timeslide_n_windows() of them.
 * The (segment, slide) work table is copied to the workspace first (this call
 * blocks until that small copy is done); all windows of all pairs then run in
 * shared batches.
 * ------------------------------------------------------------------------ */
int64_t af_timeslide_n_windows(const int64_t* seg_len, int64_t n_seg, int64_t n_slides, int64_t window,
                               int64_t stride);
size_t af_timeslide_workspace_bytes(const af_net* net, int64_t n_seg, int64_t n_slides, int64_t batch);
af_status af_score_timeslides(const af_net* net, const float* y, int64_t n_ch, int64_t ld_y, int64_t n,
                              const int64_t* seg_off, const int64_t* seg_len, int64_t n_seg,
                              const int64_t* shifts, int64_t n_slides, int64_t stride, float* logits,
                              void* ws, size_t ws_bytes, af_stream stream);

/* Two-step form for graph capture: af_timeslide_prepare copies the work table
 * into the workspace (and blocks for that copy); af_score_timeslides_prepared
 * then only enqueues kernels, so it may be captured in a graph and replayed.
 * Both take the same segments, slides, stride and workspace. */
af_status af_timeslide_prepare(const af_net* net, const int64_t* seg_off, const int64_t* seg_len, int64_t n_seg,
                               const int64_t* shifts, int64_t n_slides, int64_t stride, int64_t n,
                               void* ws, size_t ws_bytes, af_stream stream);
af_status af_score_timeslides_prepared(const af_net* net, const float* y, int64_t n_ch, int64_t ld_y, int64_t n,
                                       int64_t n_seg, int64_t n_slides, int64_t stride, int64_t n_windows,
                                       float* logits, void* ws, size_t ws_bytes, af_stream stream);

/* ------------------------------------------------------------------------
 * Graph capture (replay of launch-bound sequences).  Every library call made
 * on `stream` between begin and end is recorded (nothing runs); the graph is
 * then replayed with af_graph_launch.  Captured calls must not block (use the
 * prepared timeslide form); buffers and workspaces they use must stay
 * allocated while the graph exists.
 * ------------------------------------------------------------------------ */
typedef struct af_graph af_graph;
af_status af_graph_begin(af_stream stream);
af_status af_graph_end(af_stream stream, af_graph** out);
af_status af_graph_launch(af_graph* graph, af_stream stream);
void af_graph_destroy(af_graph* graph);

/* ------------------------------------------------------------------------
 * Integration (Sec. II: predictions integrated with a 1 s top-hat filter).
 * Causal right-aligned mean.  carry == NULL (batch), valid mode:
 *     out[i] = (1/width) sum_{j=i}^{i+width-1} p[j],  i < n - width + 1;
 * n < width writes nothing.  carry != NULL (streaming): carry is a device
 * array of width - 1 floats holding the predictions that precede p (oldest
 * first); out receives n values, out[i] = the mean of the width values of
 * carry ++ p that end at p[i], and carry is then replaced by the last
 * width - 1 values of carry ++ p.  The sums run in the batch order, so a
 * stream whose carry starts zeroed reproduces the batch values bit for bit
 * from its width-th output on, however p is chunked.  width - 1 <= 4096
 * with a carry; width == 1 needs none.
 * ------------------------------------------------------------------------ */
af_status af_integrate(const float* p, int64_t n, int64_t width, float* carry, float* out, af_stream stream);

/* ------------------------------------------------------------------------
 * Clustering (Sec. II: the integrated series is clustered so that one event
 * yields one trigger, whose detection statistic is the maximum integrated
 * value over an 8 s window).  Reading: sample i of a series is a candidate iff
 *   x[i] >  x[j] for every j in [i - half, i)   and
 *   x[i] >= x[j] for every j in (i, i + half],
 * with j limited to i's own series; so equal values resolve to the earliest,
 * candidates of one series lie more than `half` samples apart, and NaN is
 * never a candidate and blocks every candidate within half of it.
 * half = 4 s x the statistic's rate (64 at 16 Hz, 4 at 1 Hz), at most 1024.
 * x: device [n] FP32, n < 2^31.  Series s is x[off[s] .. off[s+1]) for a
 * device int64 array off[n_series + 1], non-decreasing, off[0] = 0,
 * off[n_series] = n; offsets may be NULL when n_series == 1.
 * Outputs (device): the first min(count, max_out) candidates in ascending
 * order, their sample indices in idx and values in val, and the total count
 * in *n_found (device int64).  Asynchronous on `stream`; ws (device) must
 * hold af_cluster_workspace_bytes(n).  Host-checked errors return AF_EINVAL.
 * ------------------------------------------------------------------------ */
size_t af_cluster_workspace_bytes(int64_t n);
af_status af_cluster(const float* x, int64_t n, const int64_t* offsets, int64_t n_series, int64_t half,
                     int64_t* idx, float* val, int64_t max_out, int64_t* n_found, void* ws, size_t ws_bytes,
                     af_stream stream);

/* ------------------------------------------------------------------------
 * False alarm rate (Sec. IX: the number of background (timeslide) events
 * with a detection statistic greater than the one of interest, divided by
 * the background livetime):
 *   far[q] = #{i < n_bg : bg[i] > x[q]} / livetime        (events per second)
 * bg: device [n_bg] FP32 background statistics; x: device [n_q] FP32 queries;
 * far: device [n_q] FP64.  Counts are exact (integers); the division is FP64.
 * Work is n_q x n_bg comparisons.  livetime > 0 in seconds.  Asynchronous on
 * `stream`; ws (device) must hold af_far_workspace_bytes(n_q).
 * ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------
 * Injection on the device (Sec. IV, signal injection: intrinsic polarisation
 * series are projected onto the interferometers and rescaled to a sampled
 * SNR, the total SNR of the detector network per the footnote of Sec. I).
 *
 * af_project: for injection i and detector d,
 *   out[i][d][k] = F+ hp_i(t_k - dt) + Fx hc_i(t_k - dt),  t_k = k / fs,
 * with F+ = D : e+, Fx = D : ex, D = (x x^T - y y^T)/2 from the detector's
 * arm unit vectors x, y, the polarisation tensors e+ = X X^T - Y Y^T,
 * ex = X Y^T + Y X^T of the basis X = cos(psi) e_a + sin(psi) e_d,
 * Y = -sin(psi) e_a + cos(psi) e_d around the source direction
 * s = (cos dec cos phi, cos dec sin phi, sin dec), phi = ra - gmst, with
 * e_a = (-sin phi, cos phi, 0), e_d = (-sin dec cos phi, -sin dec sin phi,
 * cos dec); and dt = -(r . s)/c for the detector vertex r (metres, Earth-
 * fixed).  hp, hc are linearly interpolated (0 outside [0, len)).  FP64
 * arithmetic, FP32 output.
 *   hp, hc: device [n_inj][len] FP32; sky: device [n_inj][4] FP64 (ra, dec,
 *   psi, gmst; radians); det: HOST [n_det][9] FP64 (vertex, x arm, y arm),
 *   1 <= n_det <= 4; out: device [n_inj][n_det][len] FP32.
 *
 * af_snr_rescale: network optimal SNR of sig[i] = [n_det][len] series,
 *   snr[i]^2 = sum_d 4 (fs/len) sum_{j : f_j >= f_low, j < len/2} |H_dj|^2 / S_d(f_j),
 *   H_dj = (1/fs) sum_k sig[i][d][k] exp(-2 pi i j k / len),  f_j = j fs/len,
 * S_d linearly interpolated on the grid m * df of psd[d] (device [n_det][n_freq]
 * FP64; bins with S <= 0 or beyond the grid skipped); then, when target
 * (device [n_inj] FP64) is not NULL and snr > 0, sig[i] *= target[i] / snr[i]
 * in place.  FP64 FFT; len a power of two in [2, 8192].  snr: device [n_inj].
 * Both asynchronous on `stream`; AF_EINVAL for host-checked errors.
 * ------------------------------------------------------------------------ */
af_status af_project(const float* hp, const float* hc, int64_t n_inj, int64_t len, double fs, const double* det,
                     int64_t n_det, const double* sky, float* out, af_stream stream);
af_status af_snr_rescale(float* sig, int64_t n_inj, int64_t n_det, int64_t len, double fs, const double* psd,
                         int64_t n_freq, double df, double f_low, const double* target, double* snr,
                         af_stream stream);

size_t af_far_workspace_bytes(int64_t n_q);
af_status af_far(const float* bg, int64_t n_bg, double livetime, const float* x, int64_t n_q, double* far,
                 void* ws, size_t ws_bytes, af_stream stream);

/* ------------------------------------------------------------------------
 * Streaming server (Sec. VI: clients stream strain to a snapshotter that keeps
 * the recent state, a whitener that estimates the PSD from the first 64 s of
 * that state, and the network; Table III: online latencies).
 *
 * Each admitted stream is an independent n_ch-detector series (n_ch = the
 * net's inputs, at most 2) pushed in host chunks of at most max_chunk samples.
 * On the device a stream keeps its recent raw strain, the PSD and whitening
 * response of its current hop, its recent whitened output and logits.  For
 * stream-relative sample a (0 = first pushed sample):
 *   PSD of hop j     = Welch over samples [j*psd_hop, j*psd_hop + psd_len)
 *   whitened y[i]    = sample psd_len + M + i, whitened with the PSD of hop
 *                      i / psd_hop (M = fduration*fs/2), produced in blocks of
 *                      `block` outputs once M samples past the block arrived
 *   logit[k]         = net(y[:, k*stride : k*stride + window])
 *   integrated[k]    = mean(logit[k .. k + integrate_width - 1])
 * which is af_psd_estimate + af_whiten + af_score_windows + af_integrate on
 * the stream's concatenated data.  Results depend only on the stream's own
 * data, not on when chunks arrive or which streams share a tick.
 *
 * af_server_tick() takes every pending chunk (up to max_tick samples per
 * stream), advances each stream, scores the new windows of all streams in one
 * batched call (continuous batching) and integrates per stream; it returns
 * when the results are in host memory.  Streams are admitted while
 * shared + (streams + 1) * per-stream bytes <= hbm_budget (AF_EBUDGET
 * otherwise); released streams free their memory for later admissions.
 * push() and poll() are thread-safe and may run concurrently with a tick;
 * admit, release and tick serialise with each other.
 * ------------------------------------------------------------------------ */
typedef struct {
    double fs;                 /* 2048                                        */
    double prescale;           /* 1e21: physical strain -> O(1)                */
    int64_t nperseg, noverlap; /* Welch segments: 4096, 2048                   */
    int64_t psd_len;           /* PSD background: 64 s                         */
    int64_t psd_hop;           /* PSD update cadence: 8 s                      */
    double fduration;          /* whitening filter length: 1 s                 */
    double highpass;           /* 32 Hz                                        */
    int64_t stride;            /* samples between windows: 128 (16 Hz)         */
    int64_t integrate_width;   /* windows per 1 s: 16                          */
    int64_t block;             /* whitening block (divides psd_hop): 2048      */
    int64_t max_chunk;         /* largest push, samples                        */
    int64_t max_tick;          /* samples per stream consumed per tick         */
    int64_t max_streams;       /* stream slots                                 */
    int64_t score_batch;       /* windows per internal scoring pass            */
    size_t hbm_budget;         /* device bytes the server may hold             */
} af_server_config;

typedef struct af_server af_server;

void af_server_default_config(af_server_config* cfg);
/* Allocates the shared state (AF_EBUDGET if it alone exceeds hbm_budget).
 * The net must outlive the server. */
af_status af_server_create(const af_net* net, const af_server_config* cfg, af_server** out);
void af_server_destroy(af_server* srv);
size_t af_server_stream_bytes(const af_server* srv);
size_t af_server_shared_bytes(const af_server* srv);
af_status af_server_admit(af_server* srv, int64_t* stream_id);
af_status af_server_release(af_server* srv, int64_t stream_id);
/* x: host [n_ch][n] float64 physical strain (copied before return). */
af_status af_server_push(af_server* srv, int64_t stream_id, const double* x, int64_t n);
/* *n_windows (may be NULL) receives the number of windows scored. */
af_status af_server_tick(af_server* srv, int64_t* n_windows);
/* Moves up to cap results to the caller (host arrays); *first_* is the index
 * of the first value returned (logit index k / integrated index k). */
af_status af_server_poll(af_server* srv, int64_t stream_id, float* logits, int64_t cap_logits,
                         int64_t* n_logits, int64_t* first_logit, float* integrated, int64_t cap_integrated,
                         int64_t* n_integrated, int64_t* first_integrated);
/* Latency from a chunk's push() to the tick that put integrated values it
 * enabled on the host: p50 / p99 in ms over all such chunks, the sample
 * count and the windows scored; reset != 0 clears them. */
af_status af_server_stats(af_server* srv, double* p50_ms, double* p99_ms, int64_t* n_samples,
                          int64_t* windows, int reset);

#ifdef __cplusplus
}
#endif
#endif /* AFRAME_MI_H */
