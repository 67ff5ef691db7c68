// Device-side injection: polarisations projected onto detectors, and the
// network optimal SNR of the projections (with rescaling to a target).
//
// Projection of injection i onto detector d (one workgroup per pair): the
// antenna patterns F+ = D : e+, Fx = D : ex of the detector tensor
// D = (x x^T - y y^T) / 2 and the wave's polarisation tensors for the sky
// position, and the delay dt = -(r . s) / c of the detector vertex r against
// the geocentre, all in FP64; each output sample is
// F+ hp(t - dt) + Fx hc(t - dt) with hp, hc linearly interpolated.
//
// SNR (one workgroup per injection): each detector's series goes through a
// radix-2 FFT in FP64 in LDS (twiddles from the FP64 table), its one-sided
// power over the PSD (linearly interpolated) is summed in a fixed order, and
// the series are scaled by target / SNR.
#include "common.h"

namespace afm {
namespace {
constexpr int INJ_NT = 256;
constexpr int SNR_NT = 256;
constexpr int SNR_MAX_LOG = 13;   // series of up to 8192 samples (128 KB of LDS)
constexpr double C_LIGHT = 299792458.0;

struct InjDet {
    double r[3], x[3], y[3];   // vertex (m), arm unit vectors, Earth-fixed
};
struct InjArgs {
    const float* hp;
    const float* hc;
    int64_t len;
    double fs;
    const double* sky;   // [n_inj][4]: ra, dec, psi, gmst
    InjDet det[4];
    int n_det;
    float* out;          // [n_inj][n_det][len]
};

__device__ __forceinline__ double interp(const float* h, int64_t len, double u) {
    const double f = floor(u);
    const int64_t i0 = (int64_t)f;
    const double w = u - f;
    const double a = (i0 >= 0 && i0 < len) ? (double)h[i0] : 0.0;
    const double b = (i0 + 1 >= 0 && i0 + 1 < len) ? (double)h[i0 + 1] : 0.0;
    return (1.0 - w) * a + w * b;
}

__global__ void __launch_bounds__(INJ_NT) project_kernel(InjArgs a) {
    const int64_t i = blockIdx.x;
    const int d = blockIdx.y;
    const double* sk = a.sky + 4 * i;
    const double phi = sk[0] - sk[3], dec = sk[1], psi = sk[2];
    const double cp = cos(phi), sp = sin(phi), cd = cos(dec), sd = sin(dec), cs = cos(psi), ss = sin(psi);
    const double s[3] = {cd * cp, cd * sp, sd};                     // toward the source
    const double ea[3] = {-sp, cp, 0.0}, ed[3] = {-sd * cp, -sd * sp, cd};
    double X[3], Y[3];
    for (int k = 0; k < 3; ++k) {
        X[k] = cs * ea[k] + ss * ed[k];
        Y[k] = -ss * ea[k] + cs * ed[k];
    }
    const InjDet& dt_ = a.det[d];
    double fp = 0.0, fx = 0.0;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            const double D = 0.5 * (dt_.x[p] * dt_.x[q] - dt_.y[p] * dt_.y[q]);
            fp += D * (X[p] * X[q] - Y[p] * Y[q]);
            fx += D * (X[p] * Y[q] + Y[p] * X[q]);
        }
    const double delay = -(dt_.r[0] * s[0] + dt_.r[1] * s[1] + dt_.r[2] * s[2]) / C_LIGHT;
    const float* hp = a.hp + i * a.len;
    const float* hc = a.hc + i * a.len;
    float* o = a.out + (i * a.n_det + d) * a.len;
    const double sh = delay * a.fs;
    for (int64_t k = threadIdx.x; k < a.len; k += INJ_NT) {
        const double u = (double)k - sh;
        o[k] = (float)(fp * interp(hp, a.len, u) + fx * interp(hc, a.len, u));
    }
}

// Bit reversal of k in `bits` bits.
__device__ __forceinline__ int brev(int k, int bits) { return (int)(__brev((unsigned)k) >> (32 - bits)); }

__global__ void __launch_bounds__(SNR_NT) snr_kernel(float* sig, int n_det, int logn, double fs,
                                                     const double* psd, int64_t n_freq, double df, double f_low,
                                                     const double* tw, const double* target, double* snr_out) {
    extern __shared__ double2 buf[];          // [n] complex
    __shared__ double red[SNR_NT];
    const int n = 1 << logn;
    const int64_t i = blockIdx.x;
    const int tid = threadIdx.x;
    double rho2 = 0.0;
    for (int d = 0; d < n_det; ++d) {
        const float* h = sig + (i * n_det + d) * (int64_t)n;
        __syncthreads();
        for (int k = tid; k < n; k += SNR_NT) buf[brev(k, logn)] = make_double2((double)h[k], 0.0);
        __syncthreads();
        for (int l = 1; l <= logn; ++l) {      // butterflies of span 2^l
            const int half = 1 << (l - 1);
            for (int b = tid; b < n / 2; b += SNR_NT) {
                const int pos = b & (half - 1), j0 = ((b >> (l - 1)) << l) + pos, j1 = j0 + half;
                const double wr = tw[2 * (pos << (logn - l))], wi = tw[2 * (pos << (logn - l)) + 1];
                const double2 u = buf[j0], v = buf[j1];
                const double vr = v.x * wr - v.y * wi, vi = v.x * wi + v.y * wr;
                buf[j0] = make_double2(u.x + vr, u.y + vi);
                buf[j1] = make_double2(u.x - vr, u.y - vi);
            }
            __syncthreads();
        }
        // 4 df_n sum |H_j|^2 / S(f_j) over f_low <= f_j, j < n/2, with H = FFT / fs
        const double dfn = fs / n;
        const double* S = psd + (int64_t)d * n_freq;
        double acc = 0.0;
        for (int j = tid; j < n / 2; j += SNR_NT) {
            const double f = j * dfn;
            if (f < f_low) continue;
            const double u = f / df;
            const int64_t m = (int64_t)floor(u);
            if (m + 1 >= n_freq) continue;       // beyond the PSD grid
            const double w = u - (double)m;
            const double Sj = (1.0 - w) * S[m] + w * S[m + 1];
            if (!(Sj > 0.0)) continue;
            const double2 H = buf[j];
            acc += (H.x * H.x + H.y * H.y) / (fs * fs) / Sj;
        }
        red[tid] = acc;
        __syncthreads();
        for (int st = SNR_NT / 2; st > 0; st >>= 1) {
            if (tid < st) red[tid] += red[tid + st];
            __syncthreads();
        }
        rho2 += 4.0 * dfn * red[0];
    }
    const double rho = sqrt(rho2);
    if (tid == 0) snr_out[i] = rho;
    if (target && rho > 0.0) {
        const float sc = (float)(target[i] / rho);
        for (int64_t k = tid; k < (int64_t)n_det * n; k += SNR_NT) sig[i * n_det * (int64_t)n + k] *= sc;
    }
}
}  // namespace
}  // namespace afm

using namespace afm;

extern "C" af_status af_project(const float* hp, const float* hc, int64_t n_inj, int64_t len, double fs,
                                const double* det, int64_t n_det, const double* sky, float* out, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(n_inj >= 0 && n_inj < (1LL << 31) && len >= 1 && fs > 0.0, "need n_inj >= 0, len >= 1, fs > 0");
    AF_CHECK_ARG(n_det >= 1 && n_det <= 4, "n_det must be in [1, 4]");
    AF_CHECK_ARG(det, "det must be non-null");
    if (n_inj == 0) return AF_OK;
    AF_CHECK_ARG(hp && hc && sky && out, "hp, hc, sky and out must be non-null");
    InjArgs a{};
    a.hp = hp; a.hc = hc; a.len = len; a.fs = fs; a.sky = sky; a.out = out; a.n_det = (int)n_det;
    for (int d = 0; d < n_det; ++d)
        for (int k = 0; k < 3; ++k) {
            a.det[d].r[k] = det[9 * d + k];
            a.det[d].x[k] = det[9 * d + 3 + k];
            a.det[d].y[k] = det[9 * d + 6 + k];
        }
    hipLaunchKernelGGL(project_kernel, dim3((unsigned)n_inj, (unsigned)n_det), dim3(INJ_NT), 0, (hipStream_t)stream,
                       a);
    AF_LAUNCHED();
    return AF_OK;
}

extern "C" af_status af_snr_rescale(float* sig, int64_t n_inj, int64_t n_det, int64_t len, double fs,
                                    const double* psd, int64_t n_freq, double df, double f_low,
                                    const double* target, double* snr, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(n_inj >= 0 && n_inj < (1LL << 31), "n_inj must be in [0, 2^31)");
    AF_CHECK_ARG(n_det >= 1 && n_det <= 4, "n_det must be in [1, 4]");
    int logn = 0;
    while ((1LL << logn) < len) ++logn;
    AF_CHECK_ARG(len >= 2 && (1LL << logn) == len && logn <= SNR_MAX_LOG, "len must be a power of two in [2, %d]",
                 1 << SNR_MAX_LOG);
    AF_CHECK_ARG(fs > 0.0 && df > 0.0 && f_low >= 0.0 && n_freq >= 2, "need fs > 0, df > 0, f_low >= 0, n_freq >= 2");
    if (n_inj == 0) return AF_OK;
    AF_CHECK_ARG(sig && psd && snr, "sig, psd and snr must be non-null");
    af_status st = ensure_tables((hipStream_t)stream);
    if (st != AF_OK) return st;
    const double* tw = twiddles_f64((int)len);
    AF_CHECK_ARG(tw, "no twiddle table for len = %lld", (long long)len);
    const size_t lds = (size_t)len * sizeof(double2);
    AF_HIP(hipFuncSetAttribute((const void*)snr_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(snr_kernel, dim3((unsigned)n_inj), dim3(SNR_NT), lds,
                       (hipStream_t)stream, sig, (int)n_det, logn, fs, psd, n_freq, df, f_low, tw, target, snr);
    AF_LAUNCHED();
    return AF_OK;
}
