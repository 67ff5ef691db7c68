// Whitening on the device.
//
// Kernel 1 (filter, FP64, one workgroup per PSD hop and detector pair):
//   A_k = 1/sqrt(S_k) above the high-pass (0 below it and where S_k <= 0),
//   q   = inverse FFT of A on the PSD's own grid (the two detectors packed as
//         real and imaginary parts: both spectra are real and even),
//   h[m]= q[m mod L] (1 + cos(pi m / M)) / 2 for |m| < M,
//   H   = FFT of h wrapped onto the 8192-point block grid; since h is real and
//         even, H0 = Re, H1 = Im of the packed transform.
//   The stored response is the pair ((H0 + H1)/2, (H0 - H1)/2) sqrt(2/fs) / 8192
//   per bin k <= 4096 (H1 = 0 for an unpaired last detector), folding in the
//   output scale and the inverse FFT's normalisation, as float.
// Kernel 2 (overlap-save, FP32, one workgroup per block of up to 6146 outputs
// and detector pair): load 8192 prescaled samples of both detectors as one
// complex sequence z, Z = FFT z, Y_k = Z_k (H0_k+H1_k)/2 + conj(Z_{N-k}) (H0_k-H1_k)/2
// (which filters the real part with H0 and the imaginary part with H1), inverse
// FFT, and keep the 8192 - 2(M-1) samples the circular wrap does not touch.
// Blocks never straddle a PSD hop, so every output uses its own hop's filter.
// The 8192-point transforms are Stockham passes of radix 32, 16, 16 with one
// butterfly (radix 32) or two (radix 16) per thread of 256: the first forward
// pass reads its inputs straight from HBM, the spectral product is applied as
// the first inverse pass reads its operands, and the last inverse pass writes
// its outputs straight to HBM.  Each pass's twiddles and the filter values
// are loaded a pass ahead of their use.
#include <atomic>
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "fft_lds.h"
#include "internal.h"

namespace afm {

constexpr int WB_LOG = 13;
constexpr int WB_N = 1 << WB_LOG;  // whitening block length

template <int LOGL, int NT>
__global__ void __launch_bounds__(NT) fir_response_kernel(
    const double* __restrict__ psd /* [n_psd][n_ch][L/2+1] */, int64_t n_ch, double fs, double highpass,
    int M, const cpx<double>* __restrict__ twL, const cpx<double>* __restrict__ twB, double out_scale,
    float2* __restrict__ resp /* [n_psd][n_pairs][WB_N/2+1] */) {
    constexpr int L = 1 << LOGL;
    constexpr int FL = L / 2 + 1;
    constexpr int FB = WB_N / 2 + 1;
    extern __shared__ unsigned char smem_raw[];
    cpx<double>* a = reinterpret_cast<cpx<double>*>(smem_raw);
    const int64_t j = blockIdx.x;
    const int64_t c0 = 2 * (int64_t)blockIdx.y;
    const bool has1 = c0 + 1 < n_ch;
    const double* s0 = psd + (j * n_ch + c0) * FL;
    const double* s1 = has1 ? s0 + FL : s0;
    {
        // all loads issued before the first use
        constexpr int PER = L / NT;
        double v0[PER], v1[PER];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int k = threadIdx.x + p * NT;
            const int kk = k <= L / 2 ? k : L - k;
            v0[p] = s0[kk];
            v1[p] = s1[kk];
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int k = threadIdx.x + p * NT;
            const int kk = k <= L / 2 ? k : L - k;
            const bool pass = (double)kk * fs / (double)L >= highpass;
            const double a0 = (pass && v0[p] > 0.0) ? 1.0 / sqrt(v0[p]) : 0.0;
            const double a1 = (has1 && pass && v1[p] > 0.0) ? 1.0 / sqrt(v1[p]) : 0.0;
            a[lds_pad(k)] = {a0, a1};
        }
    }
    __syncthreads();
    fft_lds<double, LOGL, NT>(a, twL, true);  // q = L * (q0 + i q1)
    // wrap the tapered taps onto the block grid: t = m mod WB_N, |m| < M
    constexpr int PER = WB_N / NT;
    cpx<double> g[PER];
    const double invL = 1.0 / (double)L;
    const int tstep = WB_N / (2 * M);  // M is a power of two <= L / 2
    {
        // taper cosines first (all loads in flight), then the taps
        double cs[PER];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int t = threadIdx.x + p * NT;
            const int m = t < M ? t : t - WB_N;  // tap index of position t when |m| < M
            const int am = m < 0 ? -m : m;
            // (1 + cos(pi m / M)) / 2 with cos(pi m / M) = Re exp(-2 pi i (m WB_N / 2M) / WB_N)
            cs[p] = twB[am < M ? am * tstep : 0].x;
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int t = threadIdx.x + p * NT;
            const int m = t < M ? t : t - WB_N;
            const bool tap = m > -M && m < M;
            const cpx<double> q = a[lds_pad(m & (L - 1))];  // q[m mod L]
            const double w = tap ? 0.5 * (1.0 + cs[p]) * invL : 0.0;
            g[p] = {q.x * w, q.y * w};
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) a[lds_pad(threadIdx.x + p * NT)] = g[p];
    __syncthreads();
    fft_lds<double, WB_LOG, NT>(a, twB, false);
    float2* rp = resp + (j * ((n_ch + 1) / 2) + blockIdx.y) * FB;
    for (int k = threadIdx.x; k < FB; k += NT) {
        const cpx<double> h = a[lds_pad(k)];  // (H0, H1); H1 = 0 without a second detector
        rp[k] = make_float2((float)(0.5 * (h.x + h.y) * out_scale), (float)(0.5 * (h.x - h.y) * out_scale));
    }
}

constexpr int WB_FB = WB_N / 2 + 1;
constexpr int WNT = 256;                     // threads per whitening block
constexpr int WB_LDS = WB_N + WB_N / 32;     // one pad element per 32
__device__ __forceinline__ int wpad(int i) { return i + (i >> 5); }

// Zero, in a way the compiler cannot see through: loads whose address adds
// it are neither merged with earlier loads of the same address nor hoisted
// above the point where it is made (so each pass's twiddles are loaded where
// the code says, one pass ahead of their use, and do not stay live across
// the whole kernel).
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

// Buffer resources (base address in scalar registers, byte offsets from a
// 32-bit register).  A load whose offset is out of the resource's range
// returns zero and such a store is dropped; accesses that may fall outside
// their range use the offset kOOB, which is out of range whatever immediate
// offset the compiler splits off the register offset (kOOB minus a 12-bit
// immediate still exceeds any range used here).
constexpr uint32_t kOOB = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t num_bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)num_bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    } else {
        static_assert(sizeof(T) == 4, "4- or 8-byte loads");
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    }
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
}

// Workgroup index -> block index such that the blocks one XCD runs are
// consecutive (workgroups are dealt to the 8 XCDs round robin), so that the
// 2(M-1) input samples two neighbouring blocks share are read once into that
// XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t w, int64_t G) {
    const int64_t xcd = w & 7, i = w >> 3, q = G >> 3, rem = G & 7;
    return xcd * q + (xcd < rem ? xcd : rem) + i;
}

template <typename TX>
struct WhitenArgs {
    const TX* x;
    int64_t n_ch, n, ld_x;
    float prescale_f;
    double prescale_d;
    const float2* resp;  // [n_psd][n_pairs][WB_FB] (sum, difference) pairs
    int64_t n_psd, psd_hop, blocks_per_hop, n_blocks;
    int M;
    int64_t out_start, n_out;
    const cpx<float>* tw512;  // exp(-2 pi i m / 512), m < 512
    const cpx<float>* img3;   // [15][512] exp(-2 pi i r k / 8192)
    float* y;
    int64_t ld_y;
};

// Twiddles of the radix-16 pass with span 32 for butterflies j and j + 256
// (both have k = j mod 32): w^(r k), w = exp(-2 pi i / 512).
__device__ __forceinline__ void load_t2(const cpx<float>* tw512, int j, cpx<float> (&t)[15]) {
    const __amdgpu_buffer_rsrc_t rt = rsrc(tw512 + opaque_zero(), 512 * 8);
#pragma unroll
    for (int r = 1; r < 16; ++r) t[r - 1] = bload<cpx<float>>(rt, 8u * (uint32_t)(r * (j & 31)));
}
// Twiddles of the radix-16 pass with span 512 for butterflies j + 256 q:
// exp(-2 pi i r (j + 256 q) / 8192).
__device__ __forceinline__ void load_t3(const cpx<float>* img3, int j, cpx<float> (&t)[2][15]) {
    const __amdgpu_buffer_rsrc_t rt = rsrc(img3 + opaque_zero(), 15 * 512 * 8);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 1; r < 16; ++r) t[q][r - 1] = bload<cpx<float>>(rt, 8u * (uint32_t)((r - 1) * 512 + j + 256 * q));
}

// Radix-16 Stockham pass with span 32 over the block in LDS (butterflies j
// and j + 256).
template <bool INV>
__device__ __forceinline__ void wpass_span32(cpx<float>* a, const cpx<float> (&t2)[15], int j) {
    cpx<float> v[2][16];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int bf = j + 256 * q;
        v[q][0] = a[wpad(bf)];
#pragma unroll
        for (int r = 1; r < 16; ++r) v[q][r] = cmul(a[wpad(bf + 512 * r)], INV ? cconj(t2[r - 1]) : t2[r - 1]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int bf = j + 256 * q;
        dft_reg<float, 16>(v[q], INV);
        const int base = (bf >> 5) * 512 + (bf & 31);
#pragma unroll
        for (int r = 0; r < 16; ++r) a[wpad(base + 32 * r)] = v[q][r];
    }
}

// Radix-16 Stockham pass with span 512 (the last one): butterfly bf reads
// positions bf + 512 r, and its outputs belong at the same positions.
// Leaves the results in v; no LDS writes.
template <bool INV>
__device__ __forceinline__ void wpass_span512(const cpx<float>* a, const cpx<float> (&t3)[2][15], int j,
                                              cpx<float> (&v)[2][16]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int bf = j + 256 * q;
        v[q][0] = a[wpad(bf)];
#pragma unroll
        for (int r = 1; r < 16; ++r)
            v[q][r] = cmul(a[wpad(bf + 512 * r)], INV ? cconj(t3[q][r - 1]) : t3[q][r - 1]);
        dft_reg<float, 16>(v[q], INV);
    }
}

// One workgroup per (block, detector pair).
template <typename TX>
__global__ void __launch_bounds__(WNT, 2) whiten_block_kernel(WhitenArgs<TX> A) {
    __shared__ cpx<float> a[WB_LDS];
    const int j = threadIdx.x;
    const int M = A.M;
    const int V = WB_N - 2 * (M - 1);
    // block -> (hop, first output, end of outputs)
    const int64_t b = xcd_block(blockIdx.x, A.n_blocks);
    int64_t hop, o0, o_end;
    const int64_t regular = (A.n_psd - 1) * A.blocks_per_hop;
    if (b < regular) {
        hop = b / A.blocks_per_hop;
        o0 = hop * A.psd_hop + (b % A.blocks_per_hop) * V;
        o_end = min(o0 + V, (hop + 1) * A.psd_hop);
    } else {
        hop = A.n_psd - 1;
        o0 = hop * A.psd_hop + (b - regular) * V;
        o_end = min(o0 + V, A.n_out);
    }
    const int64_t pair = blockIdx.y;
    const int64_t c0 = 2 * pair;
    const bool has1 = c0 + 1 < A.n_ch;
    const int64_t in0 = A.out_start + o0 - (M - 1);  // >= 1 by the caller's context check
    // only the inputs the block's outputs depend on: the FFT's rounding then
    // depends on nothing else (streamed and batch blocks agree bit for bit)
    const int lim = (int)min((int64_t)(o_end - o0) + 2 * (M - 1), A.n - in0);

    cpx<float> t2[15], t3[2][15];
    float2 hr[32];
    // ---- forward pass 1 (radix 32, span 1): t = j + 256 r, straight from
    // HBM; positions at or past lim read as zero ----
    {
        const TX* xb0 = A.x + c0 * A.ld_x + in0;
        const __amdgpu_buffer_rsrc_t rx0 = rsrc(xb0, (uint32_t)lim * sizeof(TX));
        const __amdgpu_buffer_rsrc_t rx1 = rsrc(has1 ? xb0 + A.ld_x : xb0, has1 ? (uint32_t)lim * sizeof(TX) : 0u);
        TX r0[32], r1[32];
#pragma unroll
        for (int r = 0; r < 32; ++r) {
            const int t = j + 256 * r;
            const uint32_t off = t < lim ? (uint32_t)t * sizeof(TX) : kOOB;
            r0[r] = bload<TX>(rx0, off);
            r1[r] = bload<TX>(rx1, off);
        }
        load_t2(A.tw512, j, t2);
        cpx<float> v[32];
#pragma unroll
        for (int r = 0; r < 32; ++r) {
            if constexpr (sizeof(TX) == 8)
                v[r] = {(float)((double)r0[r] * A.prescale_d), (float)((double)r1[r] * A.prescale_d)};
            else
                v[r] = {(float)r0[r] * A.prescale_f, (float)r1[r] * A.prescale_f};
        }
        dft_reg<float, 32>(v, false);
#pragma unroll
        for (int r = 0; r < 32; ++r) a[wpad(32 * j + r)] = v[r];
        load_t3(A.img3, j, t3);
        __syncthreads();
    }
    wpass_span32<false>(a, t2, j);
    {
        // the block's filter at k = j + 256 r (its own hop, its detector
        // pair); H is even, so bins above N/2 read bin N - k
        const __amdgpu_buffer_rsrc_t rh =
            rsrc(A.resp + (hop * ((A.n_ch + 1) / 2) + pair) * WB_FB + opaque_zero(), WB_FB * 8);
#pragma unroll
        for (int r = 0; r < 32; ++r) {
            const int k = j + 256 * r;
            hr[r] = bload<float2>(rh, 8u * (uint32_t)(k <= WB_N / 2 ? k : WB_N - k));
        }
    }
    __syncthreads();
    {
        cpx<float> v[2][16];
        wpass_span512<false>(a, t3, j, v);
        load_t2(A.tw512, j, t2);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r) a[wpad(j + 256 * q + 512 * r)] = v[q][r];
        __syncthreads();
    }

    // ---- inverse pass 1 (radix 32, span 1) with the spectral product ----
    {
        cpx<float> v[32];
#pragma unroll
        for (int r = 0; r < 32; ++r) {
            const int k = j + 256 * r;
            const cpx<float> zk = a[wpad(k)];
            const cpx<float> zn = a[wpad((WB_N - k) & (WB_N - 1))];
            v[r] = {zk.x * hr[r].x + zn.x * hr[r].y, zk.y * hr[r].x - zn.y * hr[r].y};
        }
        __syncthreads();
        dft_reg<float, 32>(v, true);
#pragma unroll
        for (int r = 0; r < 32; ++r) a[wpad(32 * j + r)] = v[r];
        load_t3(A.img3, j, t3);
        __syncthreads();
    }
    wpass_span32<true>(a, t2, j);
    __syncthreads();

    // ---- last inverse pass: outputs t = bf + 512 r go straight to HBM;
    // output o0 + u comes from position u + M - 1, and positions outside
    // [M - 1, M - 1 + cnt) are stored at kOOB and dropped ----
    cpx<float> v[2][16];
    wpass_span512<true>(a, t3, j, v);
    const int cnt = (int)(o_end - o0);
    float* yb0 = A.y + c0 * A.ld_y + o0;
    const __amdgpu_buffer_rsrc_t ry0 = rsrc(yb0, (uint32_t)cnt * 4);
    const __amdgpu_buffer_rsrc_t ry1 = rsrc(has1 ? yb0 + A.ld_y : yb0, has1 ? (uint32_t)cnt * 4 : 0u);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t u = (uint32_t)(j + 256 * q + 512 * r - (M - 1));  // wraps when negative
            const uint32_t off = u < (uint32_t)cnt ? 4u * u : kOOB;
            bstore(v[q][r].x, ry0, off);
            bstore(v[q][r].y, ry1, off);
        }
}

}  // namespace afm

using namespace afm;

namespace {
constexpr int FIR_NT = 512;
constexpr size_t FIR_LDS = (size_t)lds_padded_len(WB_N) * sizeof(cpx<double>);

template <int LOGL>
hipError_t launch_fir(const double* psd, int64_t n_ch, int64_t n_psd, double fs, double hp, int M,
                      const double* twL, const double* twB, double out_scale, float2* resp, hipStream_t s) {
    auto k = fir_response_kernel<LOGL, FIR_NT>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FIR_LDS);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)n_psd, (unsigned)((n_ch + 1) / 2));
    hipLaunchKernelGGL(k, grid, dim3(FIR_NT), FIR_LDS, s, psd, n_ch, fs, hp, M, (const cpx<double>*)twL,
                       (const cpx<double>*)twB, out_scale, resp);
    return hipGetLastError();
}
}  // namespace

size_t afm::resp_bytes_for(int64_t n_ch, int64_t n_psd) {
    return align_up((size_t)n_psd * whiten_resp_floats(n_ch) * sizeof(float), 256);
}

extern "C" size_t af_whiten_workspace_bytes(int64_t n_ch, int64_t nperseg, int64_t n_psd) {
    if (n_ch < 1 || n_psd < 1 || (nperseg != 2048 && nperseg != 4096)) return 0;
    return resp_bytes_for(n_ch, n_psd);
}

namespace afm {
// Filter responses for n_psd PSDs (FP64 build, FP32 result) into resp
// [n_psd][n_pairs][WB_N/2+1] float pairs, whiten_resp_floats(n_ch) floats per
// PSD.  Arguments are assumed validated.
af_status whiten_build_response(const double* psd, int64_t n_ch, int64_t n_psd, int64_t nperseg, double fs,
                                double highpass, int M, float* resp, hipStream_t s) {
    af_status st = ensure_tables(s);
    if (st != AF_OK) return st;
    const double* twL = twiddles_f64((int)nperseg);
    const double* twB = twiddles_f64(WB_N);
    AF_CHECK_ARG(twL && twB, "no twiddle table for nperseg = %lld", (long long)nperseg);
    const double out_scale = sqrt(2.0 / fs) / (double)WB_N;
    float2* r = (float2*)resp;
    hipError_t e = nperseg == 4096 ? launch_fir<12>(psd, n_ch, n_psd, fs, highpass, M, twL, twB, out_scale, r, s)
                                   : launch_fir<11>(psd, n_ch, n_psd, fs, highpass, M, twL, twB, out_scale, r, s);
    if (e != hipSuccess) { set_error("whitening filter launch failed: %s", hipGetErrorString(e)); return AF_EHIP; }
    return AF_OK;
}

// Overlap-save application of precomputed responses (see af_whiten).
af_status whiten_apply(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double prescale,
                       const float* resp, int64_t n_psd, int64_t psd_hop, int M, int64_t out_start, int64_t n_out,
                       float* y, int64_t ld_y, hipStream_t s) {
    af_status st = ensure_tables(s);
    if (st != AF_OK) return st;
    const float* tw512 = twiddles_f32(512);
    const float* img3 = twiddle_image_f32(WB_N, 16, 512);
    if (!tw512 || !img3) { set_error("whitening twiddle tables missing"); return AF_EHIP; }
    const int V = WB_N - 2 * (M - 1);
    if (n_psd <= 1) psd_hop = n_out;
    const int64_t bph = (psd_hop + V - 1) / V;
    const int64_t last_len = n_out - (n_psd - 1) * psd_hop;
    const int64_t n_blocks = (n_psd - 1) * bph + (last_len + V - 1) / V;
    AF_CHECK_ARG(n_blocks < (1LL << 31), "too many whitening blocks");
    dim3 grid((unsigned)n_blocks, (unsigned)((n_ch + 1) / 2));
    auto launch = [&](auto* xp) {
        using TX = std::remove_const_t<std::remove_pointer_t<decltype(xp)>>;
        WhitenArgs<TX> A{xp, n_ch, n, ld_x, (float)prescale, prescale, (const float2*)resp, n_psd, psd_hop, bph,
                         n_blocks, M, out_start, n_out, (const cpx<float>*)tw512, (const cpx<float>*)img3, y, ld_y};
        hipLaunchKernelGGL(whiten_block_kernel<TX>, grid, dim3(WNT), 0, s, A);
    };
    if (xt == AF_IN_F64)
        launch((const double*)x);
    else
        launch((const float*)x);
    AF_LAUNCHED();
    return AF_OK;
}
}  // namespace afm

namespace afm {
// M = fduration*fs/2 taps per side: a power of two with 2M <= nperseg whose
// filter leaves valid outputs in an 8192-point block.
af_status whiten_taps(double fs, double fduration, int64_t nperseg, int* M_out) {
    const double Md = fduration * fs / 2.0;
    const int M = (int)llround(Md);
    AF_CHECK_ARG(fabs(Md - M) < 1e-9 && M >= 2 && (M & (M - 1)) == 0 && 2 * M <= nperseg,
                 "fduration*fs/2 must be a power of two M with 2M <= nperseg (got %g)", Md);
    AF_CHECK_ARG(WB_N - 2 * (M - 1) > 0, "filter too long for the %d-point whitening block", WB_N);
    *M_out = M;
    return AF_OK;
}

af_status whiten_check_apply(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double prescale,
                             int64_t n_psd, int64_t psd_hop, int M, int64_t out_start, int64_t n_out, const float* y,
                             int64_t ld_y) {
    AF_CHECK_ARG(x && y, "x and y must be non-null");
    AF_CHECK_ARG(xt == AF_IN_F64 || xt == AF_IN_F32, "unknown input dtype %d", (int)xt);
    AF_CHECK_ARG(n_ch >= 1 && n >= 1 && ld_x >= n, "need n_ch >= 1, n >= 1, ld_x >= n");
    AF_CHECK_ARG(prescale > 0, "prescale must be > 0");
    AF_CHECK_ARG(n_psd >= 1, "n_psd must be >= 1");
    AF_CHECK_ARG(n_out >= 1 && ld_y >= n_out, "need n_out >= 1 and ld_y >= n_out");
    AF_CHECK_ARG(out_start >= M && out_start + n_out + M <= n,
                 "output range [%lld, %lld) needs %d samples of context on each side within n = %lld",
                 (long long)out_start, (long long)(out_start + n_out), M, (long long)n);
    if (n_psd > 1)
        AF_CHECK_ARG(psd_hop >= 1 && (n_psd - 1) * psd_hop < n_out,
                     "psd_hop must be >= 1 and every PSD hop must start inside the output");
    return AF_OK;
}
}  // namespace afm

namespace {
// What each af_whiten_response call built, by buffer address, so that
// af_whiten_apply can reject a buffer built for another filter length,
// channel count or fewer PSDs.
struct RespInfo {
    int M;
    int64_t n_ch, n_psd;
};
std::mutex g_resp_mu;
std::unordered_map<const void*, RespInfo> g_resp;

}  // namespace

extern "C" af_status af_whiten_response(const double* psd, int64_t n_ch, int64_t nperseg, int64_t n_psd, double fs,
                                        double fduration, double highpass, void* resp, size_t resp_bytes,
                                        af_stream stream) {
    clear_error();
    AF_CHECK_ARG(psd && resp, "psd and resp must be non-null");
    AF_CHECK_ARG(n_ch >= 1 && n_psd >= 1, "need n_ch >= 1 and n_psd >= 1");
    AF_CHECK_ARG(fs > 0 && highpass >= 0, "fs must be > 0 and highpass >= 0");
    AF_CHECK_ARG(nperseg == 2048 || nperseg == 4096, "nperseg must be 2048 or 4096 (got %lld)", (long long)nperseg);
    int M = 0;
    af_status st = whiten_taps(fs, fduration, nperseg, &M);
    if (st != AF_OK) return st;
    const size_t need = resp_bytes_for(n_ch, n_psd);
    AF_CHECK_ARG(resp_bytes >= need, "response buffer too small: need %zu bytes, got %zu", need, resp_bytes);
    st = whiten_build_response(psd, n_ch, n_psd, nperseg, fs, highpass, M, (float*)resp, (hipStream_t)stream);
    if (st == AF_OK) {
        std::lock_guard<std::mutex> lk(g_resp_mu);
        g_resp[resp] = RespInfo{M, n_ch, n_psd};
    }
    return st;
}

extern "C" af_status af_whiten_apply(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x, double fs,
                                     double prescale, const void* resp, size_t resp_bytes, int64_t n_psd,
                                     int64_t psd_hop, double fduration, int64_t out_start, int64_t n_out, float* y,
                                     int64_t ld_y, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(resp, "resp must be non-null");
    AF_CHECK_ARG(fs > 0, "fs must be > 0");
    int M = 0;
    af_status st = whiten_taps(fs, fduration, 4096, &M);
    if (st != AF_OK) return st;
    st = whiten_check_apply(x, xt, n_ch, n, ld_x, prescale, n_psd, psd_hop, M, out_start, n_out, y, ld_y);
    if (st != AF_OK) return st;
    const size_t need = resp_bytes_for(n_ch, n_psd);
    AF_CHECK_ARG(resp_bytes >= need, "response buffer too small: need %zu bytes, got %zu", need, resp_bytes);
    RespInfo info{0, 0, 0};
    {
        std::lock_guard<std::mutex> lk(g_resp_mu);
        auto it = g_resp.find(resp);
        AF_CHECK_ARG(it != g_resp.end(), "resp was not filled by af_whiten_response");
        info = it->second;
    }
    AF_CHECK_ARG(info.M == M, "resp holds filters of %d taps per side; fduration*fs/2 = %d", info.M, M);
    AF_CHECK_ARG(info.n_ch == n_ch && info.n_psd >= n_psd,
                 "resp holds %lld PSDs of %lld channels; asked for %lld of %lld", (long long)info.n_psd,
                 (long long)info.n_ch, (long long)n_psd, (long long)n_ch);
    return whiten_apply(x, xt, n_ch, n, ld_x, prescale, (const float*)resp, n_psd, psd_hop, M, out_start, n_out, y,
                        ld_y, (hipStream_t)stream);
}

extern "C" af_status af_whiten(const void* x, af_dtype xt, int64_t n_ch, int64_t n, int64_t ld_x,
                               double fs, double prescale, const double* psd, int64_t nperseg,
                               int64_t n_psd, int64_t psd_hop, double fduration, double highpass,
                               int64_t out_start, int64_t n_out, float* y, int64_t ld_y, void* ws,
                               size_t ws_bytes, af_stream stream) {
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
    AF_CHECK_ARG(ws && ws_bytes >= need, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    float* resp = (float*)ws;
    st = whiten_build_response(psd, n_ch, n_psd, nperseg, fs, highpass, M, resp, s);
    if (st != AF_OK) return st;
    return whiten_apply(x, xt, n_ch, n, ld_x, prescale, resp, n_psd, psd_hop, M, out_start, n_out, y, ld_y, s);
}

