// Boxcar integration of the detection statistic (1 s top hat, causal,
// right-aligned, valid mode): out[i] = (1/W) sum_{j<W} p[i+j].
#include "common.h"

namespace afm {
__global__ void integrate_kernel(const float* __restrict__ p, int64_t n_out, int width, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    float s = 0.f;
    for (int j = 0; j < width; ++j) s += p[i + j];
    out[i] = s / (float)width;
}
}  // namespace afm

using namespace afm;

extern "C" af_status af_integrate(const float* p, int64_t n, int64_t width, float* out, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(width >= 1 && width <= (1 << 20), "width must be in [1, 2^20]");
    AF_CHECK_ARG(n >= 0, "n must be >= 0");
    if (n < width) return AF_OK;
    AF_CHECK_ARG(p && out, "p and out must be non-null");
    const int64_t n_out = n - width + 1;
    hipLaunchKernelGGL(integrate_kernel, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       p, n_out, (int)width, out);
    AF_LAUNCHED();
    return AF_OK;
}
