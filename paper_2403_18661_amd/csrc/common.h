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

// ---- per-device constant tables (twiddles) ---------------------------------
// Makes sure the current device's tables are built (or being built ahead of
// later work on s); every entry point that uses a table calls it first.
// AF_EINVAL while s is capturing a graph and the tables were never built.
af_status ensure_tables(hipStream_t s);
// Device pointer to exp(-2 pi i t / n) for t < n as interleaved (re, im)
// doubles, n a power of two in [2, 8192]; null for other n or before
// ensure_tables.
const double* twiddles_f64(int n);
// exp(-2 pi i t / 512) rounded to float (n = 512 only).
const float* twiddles_f32(int n);
// Twiddles of one Stockham pass laid out in the order its butterflies use
// them: image[(r - 1) ns + k] = exp(-2 pi i r k / n) for 1 <= r < rd, k < ns,
// as interleaved float (re, im); the whitening FFT's (8192, 16, 512) only.
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
