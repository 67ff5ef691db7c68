// Whitening on the device.
//
// Kernel 1 (filter, FP64, one workgroup per PSD hop and detector pair):
//   A_k = 1/sqrt(S_k) above the high-pass (0 below it and where S_k <= 0),
//   q   = inverse FFT of A on the PSD's own grid (the two detectors packed as
//         real and imaginary parts: both spectra are real and even),
//   h[m]= q[m mod L] (1 + cos(pi m / M)) / 2 for |m| < M,
//   H   = FFT of h wrapped onto the 8192-point block grid; since h is real and
//         even, H0 = Re, H1 = Im of the packed transform.
//   The stored response is H sqrt(2/fs) / 8192, folding in the output scale and
//   the inverse FFT's normalisation, as float.
// Kernel 2 (overlap-save, FP32, one workgroup per block of up to 6146 outputs
// and detector pair): load 8192 prescaled samples of both detectors as one
// complex sequence z, Z = FFT z, Y_k = Z_k (H0_k+H1_k)/2 + conj(Z_{N-k}) (H0_k-H1_k)/2
// (which filters the real part with H0 and the imaginary part with H1), inverse
// FFT, and keep the 8192 - 2(M-1) samples the circular wrap does not touch.
// Blocks never straddle a PSD hop, so every output uses its own hop's filter.
#include "fft_lds.h"
#include "internal.h"

namespace afm {

constexpr int WB_LOG = 13;
constexpr int WB_N = 1 << WB_LOG;  // whitening block length

template <int LOGL, int NT>
__global__ void __launch_bounds__(NT) fir_response_kernel(
    const double* __restrict__ psd /* [n_psd][n_ch][L/2+1] */, int64_t n_ch, double fs, double highpass,
    int M, const cpx<double>* __restrict__ twL, const cpx<double>* __restrict__ twB, double out_scale,
    float* __restrict__ resp /* [n_psd][n_ch][WB_N/2+1] */) {
    constexpr int L = 1 << LOGL;
    constexpr int FL = L / 2 + 1;
    constexpr int FB = WB_N / 2 + 1;
    extern __shared__ unsigned char smem_raw[];
    cpx<double>* a = reinterpret_cast<cpx<double>*>(smem_raw);
    const int64_t j = blockIdx.x;
    const int64_t c0 = 2 * (int64_t)blockIdx.y;
    const bool has1 = c0 + 1 < n_ch;
    const double* s0 = psd + (j * n_ch + c0) * FL;
    const double* s1 = s0 + FL;
    for (int k = threadIdx.x; k < L; k += NT) {
        const int kk = k <= L / 2 ? k : L - k;
        const double f = (double)kk * fs / (double)L;
        const bool pass = f >= highpass;
        const double v0 = s0[kk];
        const double v1 = has1 ? s1[kk] : 0.0;
        const double a0 = (pass && v0 > 0.0) ? 1.0 / sqrt(v0) : 0.0;
        const double a1 = (pass && v1 > 0.0) ? 1.0 / sqrt(v1) : 0.0;
        a[lds_pad(k)] = {a0, a1};
    }
    __syncthreads();
    fft_lds<double, LOGL, NT>(a, twL, true);  // q = L * (q0 + i q1)
    // wrap the tapered taps onto the block grid: t = m mod WB_N, |m| < M
    constexpr int PER = WB_N / NT;
    cpx<double> g[PER];
    const double invL = 1.0 / (double)L;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int t = threadIdx.x + p * NT;
        int m = t < M ? t : (t > WB_N - M ? t - WB_N : WB_N);
        if (m == WB_N) {
            g[p] = {0.0, 0.0};
        } else {
            const int am = m < 0 ? -m : m;
            // (1 + cos(pi m / M)) / 2 with cos(pi m / M) = Re exp(-2 pi i (m WB_N / 2M) / WB_N)
            const double taper = 0.5 * (1.0 + twB[am * (WB_N / (2 * M))].x);
            cpx<double> q = a[lds_pad(((m % L) + L) % L)];
            g[p] = {q.x * invL * taper, q.y * invL * taper};
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) a[lds_pad(threadIdx.x + p * NT)] = g[p];
    __syncthreads();
    fft_lds<double, WB_LOG, NT>(a, twB, false);
    float* r0 = resp + (j * n_ch + c0) * FB;
    float* r1 = r0 + FB;
    for (int k = threadIdx.x; k < FB; k += NT) {
        cpx<double> h = a[lds_pad(k)];
        r0[k] = (float)(h.x * out_scale);
        if (has1) r1[k] = (float)(h.y * out_scale);
    }
}

template <int NT, typename TX>
__global__ void __launch_bounds__(NT) whiten_block_kernel(
    const TX* __restrict__ x, int64_t n_ch, int64_t n, int64_t ld_x, float prescale_f, double prescale_d,
    const float* __restrict__ resp, int64_t n_psd, int64_t psd_hop, int64_t blocks_per_hop, int M,
    int64_t out_start, int64_t n_out, const cpx<float>* __restrict__ tw, float* __restrict__ y, int64_t ld_y) {
    constexpr int FB = WB_N / 2 + 1;
    __shared__ cpx<float> a[lds_padded_len(WB_N)];
    const int V = WB_N - 2 * (M - 1);
    // block -> (hop, first output, end of outputs)
    const int64_t b = blockIdx.x;
    int64_t j, o0, o_end;
    const int64_t regular = (n_psd - 1) * blocks_per_hop;
    if (b < regular) {
        j = b / blocks_per_hop;
        o0 = j * psd_hop + (b % blocks_per_hop) * V;
        o_end = min(o0 + V, (j + 1) * psd_hop);
    } else {
        j = n_psd - 1;
        o0 = j * psd_hop + (b - regular) * V;
        o_end = min(o0 + V, n_out);
    }
    const int64_t c0 = 2 * (int64_t)blockIdx.y;
    const bool has1 = c0 + 1 < n_ch;
    const TX* x0 = x + c0 * ld_x;
    const TX* x1 = x + (c0 + 1) * ld_x;
    const int64_t in0 = out_start + o0 - (M - 1);
    // only the inputs the block's outputs depend on: the FFT's rounding then
    // depends on nothing else (streamed and batch blocks agree bit for bit)
    const int64_t in_len = (o_end - o0) + 2 * (M - 1);
    for (int t = threadIdx.x; t < WB_N; t += NT) {
        const int64_t p = in0 + t;
        float v0 = 0.f, v1 = 0.f;
        if (t < in_len && p < n) {
            if constexpr (sizeof(TX) == 8) {
                v0 = (float)((double)x0[p] * prescale_d);
                if (has1) v1 = (float)((double)x1[p] * prescale_d);
            } else {
                v0 = (float)x0[p] * prescale_f;
                if (has1) v1 = (float)x1[p] * prescale_f;
            }
        }
        a[lds_pad(t)] = {v0, v1};
    }
    __syncthreads();
    fft_lds<float, WB_LOG, NT>(a, tw, false);
    const float* h0 = resp + (j * n_ch + c0) * FB;
    const float* h1 = h0 + FB;
    for (int k = threadIdx.x; k <= WB_N / 2; k += NT) {
        const int kn = (WB_N - k) & (WB_N - 1);
        const float H0 = h0[k];
        const float H1 = has1 ? h1[k] : 0.f;
        const float hs = 0.5f * (H0 + H1), hd = 0.5f * (H0 - H1);
        const cpx<float> zk = a[lds_pad(k)], zn = a[lds_pad(kn)];
        const cpx<float> yk = {zk.x * hs + zn.x * hd, zk.y * hs - zn.y * hd};
        const cpx<float> yn = {zn.x * hs + zk.x * hd, zn.y * hs - zk.y * hd};
        a[lds_pad(k)] = yk;
        if (kn != k) a[lds_pad(kn)] = yn;
    }
    __syncthreads();
    fft_lds<float, WB_LOG, NT>(a, tw, true);
    float* y0 = y + c0 * ld_y;
    float* y1 = y + (c0 + 1) * ld_y;
    const int64_t cnt = o_end - o0;
    for (int q = threadIdx.x; q < cnt; q += NT) {
        const cpx<float> v = a[lds_pad(M - 1 + q)];
        y0[o0 + q] = v.x;
        if (has1) y1[o0 + q] = v.y;
    }
}

}  // namespace afm

using namespace afm;

namespace {
constexpr int FIR_NT = 512;
constexpr size_t FIR_LDS = (size_t)lds_padded_len(WB_N) * sizeof(cpx<double>);

size_t resp_bytes(int64_t n_ch, int64_t n_psd) {
    return align_up((size_t)n_psd * n_ch * (WB_N / 2 + 1) * sizeof(float), 256);
}

template <int LOGL>
hipError_t launch_fir(const double* psd, int64_t n_ch, int64_t n_psd, double fs, double hp, int M,
                      const double* twL, const double* twB, double out_scale, float* resp, hipStream_t s) {
    auto k = fir_response_kernel<LOGL, FIR_NT>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FIR_LDS);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)n_psd, (unsigned)((n_ch + 1) / 2));
    hipLaunchKernelGGL(k, grid, dim3(FIR_NT), FIR_LDS, s, psd, n_ch, fs, hp, M, (const cpx<double>*)twL,
                       (const cpx<double>*)twB, out_scale, resp);
    return hipGetLastError();
}
}  // namespace

extern "C" size_t af_whiten_workspace_bytes(int64_t n_ch, int64_t nperseg, int64_t n_psd) {
    if (n_ch < 1 || n_psd < 1 || (nperseg != 2048 && nperseg != 4096)) return 0;
    return resp_bytes(n_ch, n_psd);
}

namespace afm {
// Filter responses for n_psd PSDs (FP64 build, FP32 result) into resp
// [n_psd][n_ch][WB_N/2+1].  Arguments are assumed validated.
af_status whiten_build_response(const double* psd, int64_t n_ch, int64_t n_psd, int64_t nperseg, double fs,
                                double highpass, int M, float* resp, hipStream_t s) {
    const double* twL = twiddles_f64((int)nperseg);
    const double* twB = twiddles_f64(WB_N);
    if (!twL || !twB) { set_error("twiddle table allocation failed"); return AF_ENOMEM; }
    const double out_scale = sqrt(2.0 / fs) / (double)WB_N;
    hipError_t e = nperseg == 4096 ? launch_fir<12>(psd, n_ch, n_psd, fs, highpass, M, twL, twB, out_scale, resp, s)
                                   : launch_fir<11>(psd, n_ch, n_psd, fs, highpass, M, twL, twB, out_scale, resp, s);
    if (e != hipSuccess) { set_error("whitening filter launch failed: %s", hipGetErrorString(e)); return AF_EHIP; }
    return AF_OK;
}

// Overlap-save application of precomputed responses (see af_whiten).
af_status whiten_apply(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double prescale,
                       const float* resp, int64_t n_psd, int64_t psd_hop, int M, int64_t out_start, int64_t n_out,
                       float* y, int64_t ld_y, hipStream_t s) {
    const float* twF = twiddles_f32(WB_N);
    if (!twF) { set_error("twiddle table allocation failed"); return AF_ENOMEM; }
    const int V = WB_N - 2 * (M - 1);
    if (n_psd <= 1) psd_hop = n_out;
    const int64_t bph = (psd_hop + V - 1) / V;
    const int64_t last_len = n_out - (n_psd - 1) * psd_hop;
    const int64_t n_blocks = (n_psd - 1) * bph + (last_len + V - 1) / V;
    AF_CHECK_ARG(n_blocks < (1LL << 31), "too many whitening blocks");
    dim3 grid((unsigned)n_blocks, (unsigned)((n_ch + 1) / 2));
    if (xt == AF_IN_F64)
        hipLaunchKernelGGL((whiten_block_kernel<256, double>), grid, dim3(256), 0, s, (const double*)x, n_ch, n, ld_x,
                           (float)prescale, prescale, resp, n_psd, psd_hop, bph, M, out_start, n_out,
                           (const cpx<float>*)twF, y, ld_y);
    else
        hipLaunchKernelGGL((whiten_block_kernel<256, float>), grid, dim3(256), 0, s, (const float*)x, n_ch, n, ld_x,
                           (float)prescale, prescale, resp, n_psd, psd_hop, bph, M, out_start, n_out,
                           (const cpx<float>*)twF, y, ld_y);
    AF_LAUNCHED();
    return AF_OK;
}
}  // namespace afm

extern "C" af_status af_whiten(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x,
                               double fs, double prescale, const double* psd, int64_t nperseg,
                               int64_t n_psd, int64_t psd_hop, double fduration, double highpass,
                               int64_t out_start, int64_t n_out, float* y, int64_t ld_y, void* ws,
                               size_t ws_bytes, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(x && psd && y, "x, psd and y must be non-null");
    AF_CHECK_ARG(xt == AF_IN_F64 || xt == AF_IN_F32, "unknown input dtype %d", (int)xt);
    AF_CHECK_ARG(n_ch >= 1 && n >= 1 && ld_x >= n, "need n_ch >= 1, n >= 1, ld_x >= n");
    AF_CHECK_ARG(fs > 0 && prescale > 0 && highpass >= 0, "fs, prescale must be > 0 and highpass >= 0");
    AF_CHECK_ARG(nperseg == 2048 || nperseg == 4096, "nperseg must be 2048 or 4096 (got %lld)", (long long)nperseg);
    const double Md = fduration * fs / 2.0;
    const int M = (int)llround(Md);
    AF_CHECK_ARG(fabs(Md - M) < 1e-9 && M >= 2 && (M & (M - 1)) == 0 && 2 * M <= nperseg,
                 "fduration*fs/2 must be a power of two M with 2M <= nperseg (got %g)", Md);
    AF_CHECK_ARG(n_psd >= 1, "n_psd must be >= 1");
    AF_CHECK_ARG(n_out >= 1 && ld_y >= n_out, "need n_out >= 1 and ld_y >= n_out");
    AF_CHECK_ARG(out_start >= M && out_start + n_out + M <= n,
                 "output range [%lld, %lld) needs %d samples of context on each side within n = %lld",
                 (long long)out_start, (long long)(out_start + n_out), M, (long long)n);
    AF_CHECK_ARG(WB_N - 2 * (M - 1) > 0, "filter too long for the %d-point whitening block", WB_N);
    if (n_psd > 1)
        AF_CHECK_ARG(psd_hop >= 1 && (n_psd - 1) * psd_hop < n_out,
                     "psd_hop must be >= 1 and every PSD hop must start inside the output");
    const size_t need = resp_bytes(n_ch, n_psd);
    AF_CHECK_ARG(ws && ws_bytes >= need, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    float* resp = (float*)ws;
    af_status st = whiten_build_response(psd, n_ch, n_psd, nperseg, fs, highpass, M, resp, s);
    if (st != AF_OK) return st;
    return whiten_apply(x, xt, n_ch, n, ld_x, prescale, resp, n_psd, psd_hop, M, out_start, n_out, y, ld_y, s);
}
