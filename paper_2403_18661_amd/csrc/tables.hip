// Per-device constant tables (FFT twiddles), the library's init call and the
// thread-local error string.
//
// The twiddles exp(-2 pi i t / n) live in static device arrays, so each GPU
// holds its own copy from the moment the library's code is loaded on it and
// nothing is allocated for them.  They are computed on the device from their
// definition, cospi(-2t/n) + i sinpi(-2t/n) in FP64 (the argument -2t/n is
// exact for the power-of-two n used here), by one kernel queued on the stream
// of the first call that needs them, or eagerly by af_init.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <mutex>
#include <string>

#include "common.h"
#include "internal.h"

namespace afm {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

namespace {
constexpr int kTwMaxLog = 13;                          // FP64 tables for n = 2, 4, ..., 8192
constexpr int kTw64Cpx = (2 << kTwMaxLog) - 2;         // table n starts at complex entry n - 2
constexpr int kImgN = 8192, kImgRd = 16, kImgNs = 512; // one Stockham pass of the whitening FFT
constexpr int kTw32N = 512;

__device__ __align__(16) double g_tw64[2 * kTw64Cpx];
__device__ __align__(16) float g_tw32[2 * kTw32N];
__device__ __align__(16) float g_img[2 * (kImgRd - 1) * kImgNs];

__global__ void __launch_bounds__(256) init_tables_kernel(double* tw64, float* tw32, float* img) {
    const int stride = gridDim.x * blockDim.x;
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (int e = i0; e < kTw64Cpx; e += stride) {
        int n = 2;
        while (e >= 2 * n - 2) n <<= 1;   // e lies in table n: [n - 2, 2n - 2)
        double s, c;
        sincospi(-2.0 * (double)(e - (n - 2)) / (double)n, &s, &c);
        tw64[2 * e] = c;
        tw64[2 * e + 1] = s;
    }
    for (int t = i0; t < kTw32N; t += stride) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)kTw32N, &s, &c);
        tw32[2 * t] = (float)c;
        tw32[2 * t + 1] = (float)s;
    }
    // image[(r - 1) ns + k] = exp(-2 pi i r k / n)
    for (int e = i0; e < (kImgRd - 1) * kImgNs; e += stride) {
        const int r = e / kImgNs + 1, k = e % kImgNs;
        double s, c;
        sincospi(-2.0 * (double)((r * k) % kImgN) / (double)kImgN, &s, &c);
        img[2 * e] = (float)c;
        img[2 * e + 1] = (float)s;
    }
}

struct DevTables {
    std::atomic<int> queued{0};     // the init kernel has been enqueued
    std::atomic<int> complete{0};   // ... and has finished
    double* tw64 = nullptr;
    float* tw32 = nullptr;
    float* img = nullptr;
    hipEvent_t done = nullptr;
};
constexpr int kMaxDev = 64;
DevTables g_dev[kMaxDev];
std::mutex g_mu;

DevTables* current_tables() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
    return &g_dev[dev];
}
}  // namespace

af_status ensure_tables(hipStream_t s) {
    DevTables* T = current_tables();
    if (!T) {
        set_error("no current HIP device (or device index above %d)", kMaxDev - 1);
        return AF_EHIP;
    }
    if (T->complete.load(std::memory_order_acquire)) return AF_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    AF_HIP(hipStreamIsCapturing(s, &cs));
    if (!T->queued.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!T->queued.load(std::memory_order_relaxed)) {
            AF_CHECK_ARG(cs == hipStreamCaptureStatusNone,
                         "this device's constant tables are not built yet: call af_init() before capturing");
            AF_HIP(hipGetSymbolAddress((void**)&T->tw64, HIP_SYMBOL(g_tw64)));
            AF_HIP(hipGetSymbolAddress((void**)&T->tw32, HIP_SYMBOL(g_tw32)));
            AF_HIP(hipGetSymbolAddress((void**)&T->img, HIP_SYMBOL(g_img)));
            AF_HIP(hipEventCreateWithFlags(&T->done, hipEventDisableTiming));
            hipLaunchKernelGGL(init_tables_kernel, dim3(64), dim3(256), 0, s, T->tw64, T->tw32, T->img);
            AF_LAUNCHED();
            AF_HIP(hipEventRecord(T->done, s));
            T->queued.store(1, std::memory_order_release);
            return AF_OK;   // later work on s runs after the kernel
        }
    }
    // queued by an earlier call, maybe on another stream: wait for it on s
    const hipError_t q = hipEventQuery(T->done);
    if (q == hipSuccess) {
        T->complete.store(1, std::memory_order_release);
        return AF_OK;
    }
    if (q != hipErrorNotReady) {
        set_error("constant tables: %s", hipGetErrorString(q));
        return AF_EHIP;
    }
    AF_CHECK_ARG(cs == hipStreamCaptureStatusNone,
                 "this device's constant tables are still being built: call af_init() before capturing");
    AF_HIP(hipStreamWaitEvent(s, T->done, 0));
    return AF_OK;
}

const double* twiddles_f64(int n) {
    DevTables* T = current_tables();
    if (!T || !T->tw64 || n < 2 || n > (1 << kTwMaxLog) || (n & (n - 1))) return nullptr;
    return T->tw64 + 2 * (size_t)(n - 2);
}

const float* twiddles_f32(int n) {
    DevTables* T = current_tables();
    return T && n == kTw32N ? T->tw32 : nullptr;
}

const float* twiddle_image_f32(int n, int rd, int ns) {
    DevTables* T = current_tables();
    return T && n == kImgN && rd == kImgRd && ns == kImgNs ? T->img : nullptr;
}

}  // namespace afm

using namespace afm;

extern "C" af_status af_init(void) {
    clear_error();
    af_status st = ensure_tables(nullptr);
    if (st != AF_OK) return st;
    st = whiten_scratch_setup();
    if (st != AF_OK) return st;
    AF_HIP(hipStreamSynchronize(nullptr));
    return ensure_tables(nullptr);   // records completion
}

extern "C" const char* af_last_error(void) { return afm::last_error(); }
extern "C" const char* af_version(void) { return "aframe_mi 0.2 (gfx950)"; }
