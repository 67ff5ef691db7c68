// Shared host/device helpers of the aframe_mi library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/aframe_mi.h"

namespace afm {

// ---- host-side error plumbing -------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

#define AF_CHECK_ARG(cond, ...)                 \
    do {                                        \
        if (!(cond)) {                          \
            ::afm::set_error(__VA_ARGS__);      \
            return AF_EINVAL;                   \
        }                                       \
    } while (0)

#define AF_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::afm::set_error("%s failed: %s", #call, hipGetErrorString(e_));      \
            return AF_EHIP;                                                       \
        }                                                                         \
    } while (0)

#define AF_LAUNCHED()                                                             \
    do {                                                                          \
        hipError_t e_ = hipGetLastError();                                        \
        if (e_ != hipSuccess) {                                                   \
            ::afm::set_error("kernel launch failed: %s", hipGetErrorString(e_));  \
            return AF_EHIP;                                                       \
        }                                                                         \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---- per-device constant tables (twiddles, windows) -----------------------
// Returns a device pointer to exp(-2 pi i t / n) for t < n as interleaved
// (re, im) doubles; built on the host in FP64 on first use per device.
const double* twiddles_f64(int n);
// Same table rounded to float.
const float* twiddles_f32(int n);
// Twiddles of one Stockham pass laid out in the order its butterflies use
// them: image[(r - 1) ns + k] = exp(-2 pi i r k / n) for 1 <= r < rd, k < ns,
// as interleaved float (re, im), built in FP64 on first use per device.
const float* twiddle_image_f32(int n, int rd, int ns);

// ---- device helpers ---------------------------------------------------------
template <typename R>
struct cpx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.x, -a.y}; }

}  // namespace afm
