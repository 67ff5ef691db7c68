// Library-internal entry points shared between translation units.
#pragma once
#include "common.h"

struct af_net;

namespace afm {
af_status whiten_build_response(const double* psd, int64_t n_ch, int64_t n_psd, int64_t nperseg, double fs,
                                double highpass, int M, float* resp, hipStream_t s);
af_status whiten_apply(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double prescale,
                       const float* resp, int64_t n_psd, int64_t psd_hop, int M, int64_t out_start, int64_t n_out,
                       float* y, int64_t ld_y, hipStream_t s);
// Periodograms of n_seg segments x + i*step (FP64 physical strain times
// prescale, periodic Hann) into pg [n_seg][n_ch][nperseg/2+1].
af_status welch_pgrams(const double* x, int64_t n_ch, int64_t ld_x, double prescale, int64_t nperseg, int64_t step,
                       int64_t n_seg, double* pg, hipStream_t s);
// One-sided Welch PSD [n_ch][nperseg/2+1] from n_avg periodograms held in a
// ring of R slots starting at slot `first`, summed in segment order.
af_status welch_ring_average(const double* ring, int64_t n_ch, int64_t nperseg, int64_t R, int64_t first,
                             int64_t n_avg, double fs, double* psd, hipStream_t s);
// Score windows described by a device work table (see af_score_timeslides).
af_status score_table(const af_net* net, const float* y, int64_t ld_y, int64_t n, int64_t stride,
                      int64_t n_windows, const int64_t* table, int n_entries, float* logits, void* ws,
                      size_t ws_bytes, hipStream_t s);
int net_window(const af_net* net);
int net_in_ch(const af_net* net);
int net_device(const af_net* net);
// Looks up, once per device, the address of the static scratch array of
// af_whiten_noalloc.
af_status whiten_scratch_setup();

constexpr int kWhitenBlockOut = 6146;   // outputs per 8192-point block with a 2047-tap filter
// floats of whitening response per PSD: one (sum, difference) pair per bin of
// the 8192-point block grid for every detector pair
constexpr int64_t whiten_resp_floats(int64_t n_ch) { return ((n_ch + 1) / 2) * 2 * (8192 / 2 + 1); }
// Bytes of whitening response for n_psd PSDs of n_ch channels.
size_t resp_bytes_for(int64_t n_ch, int64_t n_psd);
// Taps per side M of a whitening filter of fduration seconds (AF_EINVAL
// unless M is a power of two with 2M <= nperseg).
af_status whiten_taps(double fs, double fduration, int64_t nperseg, int* M_out);
// Host checks of the data arguments of the whitening entry points.
af_status whiten_check_apply(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double prescale,
                             int64_t n_psd, int64_t psd_hop, int M, int64_t out_start, int64_t n_out, const float* y,
                             int64_t ld_y);
}  // namespace afm
