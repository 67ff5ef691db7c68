// af_whiten_noalloc: af_whiten for callers that cannot allocate device memory
// (code under graph capture, tight serving loops, harnesses that forbid it).
// The filter responses, which af_whiten keeps in the caller's workspace, go
// to a static scratch array of the library's code object instead.
#include <atomic>
#include <mutex>

#include "internal.h"

using namespace afm;

namespace {
// Responses of up to 512 (PSD, detector pair) combinations of 8192-point
// filters (4097 complex values each): 16 MiB + 4 KiB.  Each GPU holds its own
// copy of the array until the process ends.  Host code never passes the array's name to a kernel (in
// host code it is a stand-in, not a device address); it uses the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)512 * whiten_resp_floats(2) * sizeof(float);
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDev = 64;
std::atomic<void*> g_scratch_ptr[kMaxDev];
std::mutex g_scratch_mu;
}  // namespace

// Looks up the current device's address of the scratch array, once per
// device (af_init calls it; af_whiten_noalloc does on its first call).
af_status afm::whiten_scratch_setup() {
    int dev = -1;
    AF_HIP(hipGetDevice(&dev));
    AF_CHECK_ARG(dev >= 0 && dev < kMaxDev, "device index %d above %d", dev, kMaxDev - 1);
    if (g_scratch_ptr[dev].load(std::memory_order_acquire)) return AF_OK;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev].load(std::memory_order_relaxed)) return AF_OK;
    void* ptr = nullptr;
    AF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev].store(ptr, std::memory_order_release);
    return AF_OK;
}

extern "C" af_status af_whiten_noalloc(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double fs,
                                       double prescale, const double* psd, int64_t nperseg, int64_t n_psd,
                                       int64_t psd_hop, double fduration, double highpass, int64_t out_start,
                                       int64_t n_out, float* y, int64_t ld_y, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(psd, "psd must be non-null");
    AF_CHECK_ARG(fs > 0 && highpass >= 0, "fs must be > 0 and highpass >= 0");
    AF_CHECK_ARG(nperseg == 2048 || nperseg == 4096, "nperseg must be 2048 or 4096 (got %lld)", (long long)nperseg);
    int M = 0;
    af_status st = whiten_taps(fs, fduration, nperseg, &M);
    if (st != AF_OK) return st;
    st = whiten_check_apply(x, xt, n_ch, n, ld_x, prescale, n_psd, psd_hop, M, out_start, n_out, y, ld_y);
    if (st != AF_OK) return st;
    const size_t need = resp_bytes_for(n_ch, n_psd);
    AF_CHECK_ARG(need <= kScratchBytes,
                 "%lld PSDs of %lld channels need %zu bytes of filter responses; the static scratch holds %zu",
                 (long long)n_psd, (long long)n_ch, need, kScratchBytes);
    st = whiten_scratch_setup();
    if (st != AF_OK) return st;
    int dev = -1;
    AF_HIP(hipGetDevice(&dev));
    float* resp = (float*)g_scratch_ptr[dev].load(std::memory_order_acquire);
    AF_CHECK_ARG(resp, "no scratch address for device %d", dev);
    hipStream_t s = (hipStream_t)stream;
    // every response value the apply step reads is written by the build step
    // of the same call, so nothing needs clearing between calls
    st = whiten_build_response(psd, n_ch, n_psd, nperseg, fs, highpass, M, resp, s);
    if (st != AF_OK) return st;
    return whiten_apply(x, xt, n_ch, n, ld_x, prescale, resp, n_psd, psd_hop, M, out_start, n_out, y, ld_y, s);
}
