// Per-device constant tables and the thread-local error string.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"

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
std::mutex g_mu;
std::map<std::pair<int, int>, void*> g_tw64, g_tw32;  // (device, n) -> table
std::map<std::pair<int, long long>, void*> g_img;     // (device, packed n/rd/ns) -> table

std::vector<double> host_twiddles(int n) {
    // exp(-2 pi i t / n) evaluated in FP64 from the definition
    std::vector<double> t(2 * (size_t)n);
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < n; ++k) {
        double a = -two_pi * (double)k / (double)n;
        t[2 * k] = std::cos(a);
        t[2 * k + 1] = std::sin(a);
    }
    return t;
}
}  // namespace

const double* twiddles_f64(int n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, n);
    auto it = g_tw64.find(key);
    if (it != g_tw64.end()) return (const double*)it->second;
    std::vector<double> h = host_twiddles(n);
    void* d = nullptr;
    if (hipMalloc(&d, h.size() * sizeof(double)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    g_tw64[key] = d;
    return (const double*)d;
}

const float* twiddles_f32(int n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, n);
    auto it = g_tw32.find(key);
    if (it != g_tw32.end()) return (const float*)it->second;
    std::vector<double> h = host_twiddles(n);
    std::vector<float> f(h.size());
    for (size_t i = 0; i < h.size(); ++i) f[i] = (float)h[i];
    void* d = nullptr;
    if (hipMalloc(&d, f.size() * sizeof(float)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    g_tw32[key] = d;
    return (const float*)d;
}

const float* twiddle_image_f32(int n, int rd, int ns) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, ((long long)n << 32) | ((long long)rd << 16) | (long long)ns);
    auto it = g_img.find(key);
    if (it != g_img.end()) return (const float*)it->second;
    // image[(r - 1) ns + k] = exp(-2 pi i r k / n), from the definition in FP64
    const double two_pi = 6.283185307179586476925286766559;
    std::vector<float> f(2 * (size_t)(rd - 1) * ns);
    for (int r = 1; r < rd; ++r)
        for (int k = 0; k < ns; ++k) {
            const long long m = ((long long)r * k) % n;
            const double a = -two_pi * (double)m / (double)n;
            const size_t i = 2 * ((size_t)(r - 1) * ns + k);
            f[i] = (float)std::cos(a);
            f[i + 1] = (float)std::sin(a);
        }
    void* d = nullptr;
    if (hipMalloc(&d, f.size() * sizeof(float)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    g_img[key] = d;
    return (const float*)d;
}

}  // namespace afm

extern "C" const char* af_last_error(void) { return afm::last_error(); }
extern "C" const char* af_version(void) { return "aframe_mi 0.1 (gfx950)"; }
