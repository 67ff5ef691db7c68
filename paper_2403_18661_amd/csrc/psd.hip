// Welch PSD on the device, FP64 throughout.
//
// Kernel 1 (periodograms): one workgroup per (segment, detector pair).  The
// two detectors' windowed segments are packed as the real and imaginary parts
// of one complex sequence, transformed by one in-LDS FFT, and separated with
// X0_k = (Z_k + conj Z_{N-k}) / 2, X1_k = (Z_k - conj Z_{N-k}) / (2i).
// Segments sit on one global grid (step nperseg - noverlap), so a rolling
// background shares every segment spectrum between the PSDs that contain it.
// Kernel 2 (average): PSD_j[c][k] = c_k / (fs sum w^2) * mean of the S
// periodograms of background j, summed in segment order.
#include <cmath>

#include "fft_lds.h"
#include "internal.h"

namespace afm {

template <int LOGN, int NT, typename TX>
__global__ void __launch_bounds__(NT) welch_periodogram_kernel(
    const TX* __restrict__ x, int64_t n_ch, int64_t ld_x, double prescale, int64_t step,
    const cpx<double>* __restrict__ tw, double* __restrict__ pgram /* [G][n_ch][F] */) {
    constexpr int N = 1 << LOGN;
    constexpr int F = N / 2 + 1;
    __shared__ cpx<double> a[lds_padded_len(N)];
    const int64_t g = blockIdx.x;
    const int64_t c0 = 2 * (int64_t)blockIdx.y;
    const bool has1 = c0 + 1 < n_ch;
    const TX* x0 = x + c0 * ld_x + g * step;
    const TX* x1 = has1 ? x0 + ld_x : x0;
    {
        // all loads issued before the first use
        constexpr int PER = N / NT;
        TX u0[PER], u1[PER];
        double c[PER];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int t = threadIdx.x + p * NT;
            u0[p] = x0[t];
            u1[p] = x1[t];
            c[p] = tw[t].x;  // cos(2 pi t / N)
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const double w = 0.5 - 0.5 * c[p];  // periodic Hann
            a[lds_pad(threadIdx.x + p * NT)] = {(double)u0[p] * prescale * w,
                                                has1 ? (double)u1[p] * prescale * w : 0.0};
        }
    }
    __syncthreads();
    fft_lds<double, LOGN, NT>(a, tw, false);
    double* p0 = pgram + (g * n_ch + c0) * F;
    double* p1 = p0 + F;
    for (int k = threadIdx.x; k < F; k += NT) {
        cpx<double> zk = a[lds_pad(k)];
        cpx<double> zn = a[lds_pad((N - k) & (N - 1))];
        const double sr = zk.x + zn.x, si = zk.y - zn.y;  // Z_k + conj Z_{N-k}
        const double dr = zk.x - zn.x, di = zk.y + zn.y;  // Z_k - conj Z_{N-k}
        p0[k] = 0.25 * (sr * sr + si * si);
        if (has1) p1[k] = 0.25 * (dr * dr + di * di);
    }
}

__global__ void welch_average_kernel(const double* __restrict__ pgram, int64_t n_ch, int F,
                                     int64_t n_psd, int64_t hop_seg, int64_t n_avg, double scale,
                                     double* __restrict__ psd /* [n_psd][n_ch][F] */) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = n_psd * n_ch * F;
    if (idx >= total) return;
    const int k = (int)(idx % F);
    const int64_t c = (idx / F) % n_ch;
    const int64_t j = idx / ((int64_t)F * n_ch);
    const double* p = pgram + ((j * hop_seg) * n_ch + c) * F + k;
    const int64_t stride = n_ch * (int64_t)F;
    // summed in segment order; loads issued 16 at a time ahead of the sums
    double s = 0.0;
    int64_t i = 0;
    for (; i + 16 <= n_avg; i += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = p[(i + u) * stride];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
    }
    for (; i < n_avg; ++i) s += p[i * stride];
    const double ck = (k == 0 || k == F - 1) ? 1.0 : 2.0;
    psd[idx] = s / (double)n_avg * scale * ck;
}

// Mean of n_avg periodograms held in a ring of R slots ([R][n_ch][F]),
// starting at slot `first`, summed in segment order (the order
// welch_average_kernel sums a contiguous run in).
__global__ void welch_ring_average_kernel(const double* __restrict__ ring, int64_t n_ch, int F, int64_t R,
                                          int64_t first, int64_t n_avg, double scale, double* __restrict__ psd) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_ch * F) return;
    const int k = (int)(idx % F);
    const int64_t stride = n_ch * (int64_t)F;
    double s = 0.0;
    for (int64_t i = 0; i < n_avg; ++i) {
        int64_t slot = first + i;
        if (slot >= R) slot -= R;
        s += ring[slot * stride + idx];
    }
    const double ck = (k == 0 || k == F - 1) ? 1.0 : 2.0;
    psd[idx] = s / (double)n_avg * scale * ck;
}

}  // namespace afm

using namespace afm;

namespace {
struct WelchGeom {
    int64_t step, n_avg, hop_seg, n_seg_total;
    int F;
};

bool welch_geom(int64_t n, int64_t nperseg, int64_t noverlap, int64_t psd_len, int64_t psd_hop,
                int64_t n_psd, WelchGeom* g) {
    if (nperseg < 256 || nperseg > 4096 || (nperseg & (nperseg - 1))) {
        set_error("nperseg must be a power of two in [256, 4096] (got %lld)", (long long)nperseg);
        return false;
    }
    if (noverlap < 0 || noverlap >= nperseg) {
        set_error("noverlap must be in [0, nperseg)");
        return false;
    }
    if (n_psd < 1 || psd_len < nperseg) {
        set_error("need n_psd >= 1 and psd_len >= nperseg");
        return false;
    }
    g->step = nperseg - noverlap;
    g->n_avg = (psd_len - nperseg) / g->step + 1;
    g->F = (int)(nperseg / 2 + 1);
    if (n_psd > 1) {
        if (psd_hop <= 0 || psd_hop % g->step != 0) {
            set_error("psd_hop must be a positive multiple of nperseg - noverlap when n_psd > 1");
            return false;
        }
        g->hop_seg = psd_hop / g->step;
    } else {
        g->hop_seg = 0;
    }
    g->n_seg_total = (n_psd - 1) * g->hop_seg + g->n_avg;
    if (n >= 0) {
        const int64_t need = (n_psd - 1) * (n_psd > 1 ? psd_hop : 0) + psd_len;
        if (need > n) {
            set_error("PSD backgrounds need %lld samples but n = %lld", (long long)need, (long long)n);
            return false;
        }
    }
    return true;
}

template <int LOGN, typename TX>
void launch_pgram(const void* x, int64_t n_ch, int64_t ld_x, double prescale, int64_t step,
                  int64_t G, const double* tw, double* pg, hipStream_t s) {
    dim3 grid((unsigned)G, (unsigned)((n_ch + 1) / 2));
    hipLaunchKernelGGL((welch_periodogram_kernel<LOGN, 256, TX>), grid, dim3(256), 0, s,
                       (const TX*)x, n_ch, ld_x, prescale, step, (const cpx<double>*)tw, pg);
}

template <typename TX>
void dispatch_pgram(int logn, const void* x, int64_t n_ch, int64_t ld_x, double prescale,
                    int64_t step, int64_t G, const double* tw, double* pg, hipStream_t s) {
    switch (logn) {
        case 8: launch_pgram<8, TX>(x, n_ch, ld_x, prescale, step, G, tw, pg, s); break;
        case 9: launch_pgram<9, TX>(x, n_ch, ld_x, prescale, step, G, tw, pg, s); break;
        case 10: launch_pgram<10, TX>(x, n_ch, ld_x, prescale, step, G, tw, pg, s); break;
        case 11: launch_pgram<11, TX>(x, n_ch, ld_x, prescale, step, G, tw, pg, s); break;
        default: launch_pgram<12, TX>(x, n_ch, ld_x, prescale, step, G, tw, pg, s); break;
    }
}

// 1 / (fs sum w^2) for the periodic Hann window, from its definition
double welch_density_scale(double fs, int64_t nperseg) {
    double sw2 = 0.0;
    for (int64_t t = 0; t < nperseg; ++t) {
        const double w = 0.5 - 0.5 * std::cos(6.283185307179586476925286766559 * (double)t / (double)nperseg);
        sw2 += w * w;
    }
    return 1.0 / (fs * sw2);
}
}  // namespace

namespace afm {
af_status welch_pgrams(const double* x, int64_t n_ch, int64_t ld_x, double prescale, int64_t nperseg, int64_t step,
                       int64_t n_seg, double* pg, hipStream_t s) {
    if (n_seg <= 0) return AF_OK;
    af_status st = ensure_tables(s);
    if (st != AF_OK) return st;
    const double* tw = twiddles_f64((int)nperseg);
    AF_CHECK_ARG(tw && nperseg >= 256, "no twiddle table for nperseg = %lld", (long long)nperseg);
    int logn = 0;
    while ((1LL << logn) < nperseg) ++logn;
    dispatch_pgram<double>(logn, x, n_ch, ld_x, prescale, step, n_seg, tw, pg, s);
    AF_LAUNCHED();
    return AF_OK;
}

af_status welch_ring_average(const double* ring, int64_t n_ch, int64_t nperseg, int64_t R, int64_t first,
                             int64_t n_avg, double fs, double* psd, hipStream_t s) {
    const int F = (int)(nperseg / 2 + 1);
    const int64_t total = n_ch * F;
    hipLaunchKernelGGL(welch_ring_average_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ring, n_ch,
                       F, R, first, n_avg, welch_density_scale(fs, nperseg), psd);
    AF_LAUNCHED();
    return AF_OK;
}
}  // namespace afm

extern "C" size_t af_psd_workspace_bytes(int64_t n_ch, int64_t nperseg, int64_t noverlap,
                                         int64_t psd_len, int64_t psd_hop, int64_t n_psd) {
    WelchGeom g;
    if (n_ch < 1 || !welch_geom(-1, nperseg, noverlap, psd_len, psd_hop, n_psd, &g)) return 0;
    return align_up((size_t)g.n_seg_total * n_ch * g.F * sizeof(double), 256);
}

extern "C" af_status af_psd_estimate(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x,
                                     double fs, double prescale, int64_t nperseg, int64_t noverlap,
                                     int64_t psd_len, int64_t psd_hop, int64_t n_psd, double* psd,
                                     void* ws, size_t ws_bytes, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(x && psd, "x and psd must be non-null");
    AF_CHECK_ARG(xt == AF_IN_F64 || xt == AF_IN_F32, "unknown input dtype %d", (int)xt);
    AF_CHECK_ARG(n_ch >= 1 && n >= 1 && ld_x >= n, "need n_ch >= 1, n >= 1, ld_x >= n");
    AF_CHECK_ARG(fs > 0 && prescale > 0, "fs and prescale must be positive");
    WelchGeom g;
    if (!welch_geom(n, nperseg, noverlap, psd_len, psd_hop, n_psd, &g)) return AF_EINVAL;
    const size_t need = af_psd_workspace_bytes(n_ch, nperseg, noverlap, psd_len, psd_hop, n_psd);
    AF_CHECK_ARG(ws && ws_bytes >= need, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
    AF_CHECK_ARG(g.n_seg_total < (1LL << 31), "too many segments");
    hipStream_t s = (hipStream_t)stream;
    af_status st = ensure_tables(s);
    if (st != AF_OK) return st;
    const double* tw = twiddles_f64((int)nperseg);
    AF_CHECK_ARG(tw, "no twiddle table for nperseg = %lld", (long long)nperseg);
    int logn = 0;
    while ((1LL << logn) < nperseg) ++logn;
    double* pg = (double*)ws;
    if (xt == AF_IN_F64)
        dispatch_pgram<double>(logn, x, n_ch, ld_x, prescale, g.step, g.n_seg_total, tw, pg, s);
    else
        dispatch_pgram<float>(logn, x, n_ch, ld_x, prescale, g.step, g.n_seg_total, tw, pg, s);
    AF_LAUNCHED();
    const int64_t total = n_psd * n_ch * g.F;
    hipLaunchKernelGGL(welch_average_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       pg, n_ch, g.F, n_psd, g.hop_seg, g.n_avg, welch_density_scale(fs, nperseg), psd);
    AF_LAUNCHED();
    return AF_OK;
}
