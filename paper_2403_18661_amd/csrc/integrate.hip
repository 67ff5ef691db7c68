// Boxcar integration of the detection statistic (1 s top hat, causal,
// right-aligned): out[i] = (1/W) sum_{j<W} p[i+j] in valid mode, or, with a
// carry of the W - 1 predictions that precede p (streaming), one output per
// new prediction.
#include "common.h"

namespace afm {
__global__ void integrate_kernel(const float* __restrict__ p, int64_t n_out, int width, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    float s = 0.f;
    for (int j = 0; j < width; ++j) s += p[i + j];
    out[i] = s / (float)width;
}

// out[i] averages the W values of carry ++ p that end at p[i], summed in the
// same order as integrate_kernel sums them, so a stream reproduces the batch
// values bit for bit.
__global__ void integrate_carry_kernel(const float* __restrict__ p, int64_t n, int width,
                                       const float* __restrict__ carry, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int j = 0; j < width; ++j) {
        const int64_t k = i + j - (width - 1);   // index into p; negative reaches back into carry
        s += k >= 0 ? p[k] : carry[width - 1 + k];
    }
    out[i] = s / (float)width;
}

// carry <- the last W - 1 values of carry ++ p.  One workgroup: every value is
// read into registers before any is written, so the shift may overlap itself.
constexpr int kCarryNT = 1024, kCarryPer = 4;   // W - 1 <= 4096
__global__ void __launch_bounds__(kCarryNT) carry_update_kernel(const float* __restrict__ p, int64_t n, int width,
                                                               float* carry) {
    const int keep = width - 1;
    float v[kCarryPer];
#pragma unroll
    for (int u = 0; u < kCarryPer; ++u) {
        const int m = threadIdx.x + u * kCarryNT;
        const int64_t k = n + m;               // index into carry ++ p
        v[u] = m < keep ? (k < keep ? carry[k] : p[k - keep]) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kCarryPer; ++u) {
        const int m = threadIdx.x + u * kCarryNT;
        if (m < keep) carry[m] = v[u];
    }
}
}  // namespace afm

using namespace afm;

extern "C" af_status af_integrate(const float* p, int64_t n, int64_t width, float* carry, float* out,
                                  af_stream stream) {
    clear_error();
    AF_CHECK_ARG(width >= 1 && width <= (1 << 20), "width must be in [1, 2^20]");
    AF_CHECK_ARG(n >= 0, "n must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (carry || width == 1) {
        if (width > 1) AF_CHECK_ARG(width - 1 <= kCarryNT * kCarryPer, "a carry holds at most %d values",
                                    kCarryNT * kCarryPer);
        if (n == 0) return AF_OK;
        AF_CHECK_ARG(p && out, "p and out must be non-null");
        if (width == 1 && !carry) {
            hipLaunchKernelGGL(integrate_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, 1, out);
            AF_LAUNCHED();
            return AF_OK;
        }
        hipLaunchKernelGGL(integrate_carry_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n,
                           (int)width, (const float*)carry, out);
        AF_LAUNCHED();
        if (width > 1) {
            hipLaunchKernelGGL(carry_update_kernel, dim3(1), dim3(kCarryNT), 0, s, p, n, (int)width, carry);
            AF_LAUNCHED();
        }
        return AF_OK;
    }
    if (n < width) return AF_OK;
    AF_CHECK_ARG(p && out, "p and out must be non-null");
    const int64_t n_out = n - width + 1;
    hipLaunchKernelGGL(integrate_kernel, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, s,
                       p, n_out, (int)width, out);
    AF_LAUNCHED();
    return AF_OK;
}
