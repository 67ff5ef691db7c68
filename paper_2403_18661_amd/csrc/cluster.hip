// Candidate events and false alarm rates from the integrated statistic.
//
// Clustering: sample i of a series is a candidate iff it is larger than every
// sample up to `half` before it and at least as large as every sample up to
// `half` after it, within its own series (one trigger per excursion, the
// maximum over the window as its detection statistic).  Three kernels: a
// per-sample window test over an LDS tile with per-block counts, one scan of
// the counts, and an ordered scatter, so the candidate list is deterministic
// and ascending.
//
// False alarm rate of a statistic x: the number of background candidates
// above x divided by the background livetime.  Exact integer counts over a
// 2-D grid of (query tile, background chunk) with integer atomics.
#include "common.h"

namespace afm {
namespace {
constexpr int CL_NT = 256;
constexpr int CL_MAX_HALF = 1024;
constexpr int FAR_NT = 256;
constexpr int FAR_TILE = 2048;
constexpr int64_t FAR_CHUNK = 1 << 16;   // background values per blockIdx.y

// Bounds [lo, hi) of the series holding sample i: the largest s with off[s] <= i.
__device__ __forceinline__ void series_bounds(const int64_t* off, int n_series, int64_t i, int64_t& lo, int64_t& hi) {
    int a = 0, b = n_series - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (off[m] <= i) a = m; else b = m - 1;
    }
    lo = off[a];
    hi = off[a + 1];
}

__global__ void __launch_bounds__(CL_NT) cluster_flag_kernel(const float* __restrict__ x, int64_t n,
                                                             const int64_t* __restrict__ off, int n_series, int half,
                                                             uint8_t* __restrict__ flag, int* __restrict__ blk_count) {
    __shared__ float tile[CL_NT + 2 * CL_MAX_HALF];   // samples b0 - half ... b0 + CL_NT + half
    const int64_t b0 = (int64_t)blockIdx.x * CL_NT;
    for (int k = threadIdx.x; k < CL_NT + 2 * half; k += CL_NT) {
        const int64_t j = b0 - half + k;
        tile[k] = (j >= 0 && j < n) ? x[j] : 0.f;   // entries outside [0, n) are never compared
    }
    __syncthreads();
    const int64_t i = b0 + threadIdx.x;
    int is = 0;
    if (i < n) {
        int64_t lo = 0, hi = n;
        if (off) series_bounds(off, n_series, i, lo, hi);
        const float v = tile[threadIdx.x + half];
        is = 1;
        // j - b0 + half stays in [0, CL_NT + 2 half): |j - i| <= half
        for (int64_t j = (i - half > lo ? i - half : lo); j < i; ++j)
            if (!(tile[j - b0 + half] < v)) { is = 0; break; }
        const int64_t je = (i + half < hi - 1 ? i + half : hi - 1);
        if (is)
            for (int64_t j = i + 1; j <= je; ++j)
                if (!(tile[j - b0 + half] <= v)) { is = 0; break; }
        flag[i] = (uint8_t)is;
    }
    const int c = __syncthreads_count(is);
    if (threadIdx.x == 0) blk_count[blockIdx.x] = c;
}

// Exclusive scan of the per-block counts, in place, by one workgroup; the
// total goes to *n_found.
__global__ void __launch_bounds__(1024) cluster_scan_kernel(int* __restrict__ blk, int nb,
                                                           int64_t* __restrict__ n_found) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int a = t * per < nb ? t * per : nb, e = a + per < nb ? a + per : nb;
    int64_t s = 0;
    for (int k = a; k < e; ++k) s += blk[k];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int k = a; k < e; ++k) {
        const int c = blk[k];
        blk[k] = (int)run;
        run += c;
    }
    if (t == 1023) *n_found = part[1023];
}

__global__ void __launch_bounds__(CL_NT) cluster_scatter_kernel(const float* __restrict__ x, int64_t n,
                                                                const uint8_t* __restrict__ flag,
                                                                const int* __restrict__ blk_off,
                                                                int64_t* __restrict__ idx, float* __restrict__ val,
                                                                int64_t max_out) {
    __shared__ int wcnt[CL_NT / 64];
    const int64_t i = (int64_t)blockIdx.x * CL_NT + threadIdx.x;
    const int is = i < n ? flag[i] : 0;
    const uint64_t m = __ballot(is);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wcnt[w] = __popcll(m);
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; ++k) woff += wcnt[k];
    if (is) {
        const int64_t pos = (int64_t)blk_off[blockIdx.x] + woff + __popcll(m & ((1ull << lane) - 1ull));
        if (pos < max_out) {
            idx[pos] = i;
            val[pos] = x[i];
        }
    }
}

__global__ void __launch_bounds__(256) fill_u64_kernel(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// cnt[q] += #{background values of chunk blockIdx.y greater than x[q]}
__global__ void __launch_bounds__(FAR_NT) far_count_kernel(const float* __restrict__ bg, int64_t n_bg,
                                                           const float* __restrict__ q, int64_t n_q,
                                                           unsigned long long* __restrict__ cnt) {
    __shared__ float tile[FAR_TILE];
    const int64_t k = (int64_t)blockIdx.x * FAR_NT + threadIdx.x;
    const float xq = k < n_q ? q[k] : 0.f;
    const int64_t c0 = (int64_t)blockIdx.y * FAR_CHUNK;
    const int64_t c1 = c0 + FAR_CHUNK < n_bg ? c0 + FAR_CHUNK : n_bg;
    unsigned long long c = 0;
    for (int64_t t0 = c0; t0 < c1; t0 += FAR_TILE) {
        const int m = (int)(c1 - t0 < FAR_TILE ? c1 - t0 : FAR_TILE);
        __syncthreads();
        for (int e = threadIdx.x; e < m; e += FAR_NT) tile[e] = bg[t0 + e];
        __syncthreads();
        int cc = 0;
        for (int e = 0; e < m; ++e) cc += tile[e] > xq;
        c += (unsigned long long)cc;
    }
    if (k < n_q && c) atomicAdd(&cnt[k], c);
}

__global__ void __launch_bounds__(256) far_finish_kernel(const unsigned long long* __restrict__ cnt, int64_t n_q,
                                                         double livetime, double* __restrict__ far) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n_q) far[k] = (double)cnt[k] / livetime;
}
}  // namespace
}  // namespace afm

using namespace afm;

extern "C" size_t af_cluster_workspace_bytes(int64_t n) {
    if (n < 0) return 0;
    const int64_t nb = (n + CL_NT - 1) / CL_NT;
    return (size_t)((n + 255) / 256 * 256) + (size_t)nb * sizeof(int) + 256;
}

extern "C" af_status af_cluster(const float* x, int64_t n, const int64_t* offsets, int64_t n_series, int64_t half,
                                int64_t* idx, float* val, int64_t max_out, int64_t* n_found, void* ws,
                                size_t ws_bytes, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(n >= 0 && n < (1LL << 31), "n must be in [0, 2^31)");
    AF_CHECK_ARG(half >= 0 && half <= CL_MAX_HALF, "half must be in [0, %d]", CL_MAX_HALF);
    AF_CHECK_ARG(n_series >= 1 && n_series < (1LL << 31), "n_series must be in [1, 2^31)");
    AF_CHECK_ARG(offsets || n_series == 1, "offsets may be null only for a single series");
    AF_CHECK_ARG(max_out >= 0, "max_out must be >= 0");
    AF_CHECK_ARG(n_found, "n_found must be non-null");
    AF_CHECK_ARG(max_out == 0 || (idx && val), "idx and val must be non-null when max_out > 0");
    AF_CHECK_ARG(ws && ws_bytes >= af_cluster_workspace_bytes(n), "workspace too small: need %zu bytes",
                 af_cluster_workspace_bytes(n));
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {   // a kernel, not a memset, so that the call can be captured in a graph
        hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(256), 0, s, (unsigned long long*)n_found, (int64_t)1);
        AF_LAUNCHED();
        return AF_OK;
    }
    const int64_t nb = (n + CL_NT - 1) / CL_NT;
    uint8_t* flag = (uint8_t*)ws;
    int* blk = (int*)((char*)ws + (n + 255) / 256 * 256);
    hipLaunchKernelGGL(cluster_flag_kernel, dim3((unsigned)nb), dim3(CL_NT), 0, s, x, n, offsets, (int)n_series,
                       (int)half, flag, blk);
    hipLaunchKernelGGL(cluster_scan_kernel, dim3(1), dim3(1024), 0, s, blk, (int)nb, n_found);
    hipLaunchKernelGGL(cluster_scatter_kernel, dim3((unsigned)nb), dim3(CL_NT), 0, s, x, n, flag, blk, idx, val,
                       max_out);
    AF_LAUNCHED();
    return AF_OK;
}

extern "C" size_t af_far_workspace_bytes(int64_t n_q) { return n_q > 0 ? (size_t)n_q * 8 + 256 : 256; }

extern "C" af_status af_far(const float* bg, int64_t n_bg, double livetime, const float* x, int64_t n_q,
                            double* far, void* ws, size_t ws_bytes, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(n_bg >= 0 && n_q >= 0, "n_bg and n_q must be >= 0");
    AF_CHECK_ARG(livetime > 0.0, "livetime must be positive");
    AF_CHECK_ARG(n_q < (1LL << 40) && n_bg < (1LL << 40), "sizes too large");
    if (n_q == 0) return AF_OK;
    AF_CHECK_ARG(x && far && (bg || n_bg == 0), "x, far and bg must be non-null");
    AF_CHECK_ARG(ws && ws_bytes >= af_far_workspace_bytes(n_q), "workspace too small: need %zu bytes",
                 af_far_workspace_bytes(n_q));
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* cnt = (unsigned long long*)ws;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n_q + 255) / 256)), dim3(256), 0, s, cnt, n_q);
    if (n_bg > 0) {
        const int64_t gy = (n_bg + FAR_CHUNK - 1) / FAR_CHUNK;
        AF_CHECK_ARG(gy < 65536 && (n_q + FAR_NT - 1) / FAR_NT < (1LL << 31), "sizes too large");
        hipLaunchKernelGGL(far_count_kernel, dim3((unsigned)((n_q + FAR_NT - 1) / FAR_NT), (unsigned)gy), dim3(FAR_NT),
                           0, s, bg, n_bg, x, n_q, cnt);
    }
    hipLaunchKernelGGL(far_finish_kernel, dim3((unsigned)((n_q + 255) / 256)), dim3(256), 0, s, cnt, n_q, livetime,
                       far);
    AF_LAUNCHED();
    return AF_OK;
}
