// Device kernels of the scoring network: stem, implicit-GEMM MFMA convolution,
// global-average-pool + FC head.  Activations are stored channels-last,
// [window][time][channel], so that for a conv of kernel KW and stride S the
// implicit-GEMM row for output time t reads the contiguous input rows
// t*S - (KW-1)/2 ... t*S + (KW-1)/2 of the window.
#pragma once
#include "common.h"

namespace afm {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---- scalar conversions -----------------------------------------------------
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    // round to nearest even (inputs are finite)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
// FP32 -> OCP E4M3, round to nearest even, saturating at +-448.
__device__ __forceinline__ uint8_t f32_to_e4m3(float v) {
    const uint32_t u = __float_as_uint(v);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    const float a = fabsf(v);
    if (!(a < 448.f)) return sign | 0x7E;
    if (a < 0.015625f) {                        // below 2^-6: subnormal step 2^-9
        const int q = (int)rintf(a * 512.f);    // exact scaling, rintf rounds half to even
        return sign | (uint8_t)q;               // q == 8 is the smallest normal, 0x08
    }
    const uint32_t ua = __float_as_uint(a);
    int e = (int)(ua >> 23) - 127;
    const uint32_t mant = ua & 0x7FFFFFu;
    uint32_t m3 = (mant + 0x7FFFFu + ((mant >> 20) & 1u)) >> 20;
    if (m3 == 8u) { m3 = 0u; e += 1; }
    if (e > 8 || (e == 8 && m3 > 6u)) return sign | 0x7E;
    return sign | (uint8_t)(((e + 7) << 3) | (int)m3);
}

// ---- precision traits -----------------------------------------------------------
// Act: stored activation element; Op: LDS operand element; KL: k values per
// lane per MFMA; MK = 4 KL: k per MFMA (16x16xMK).
struct PF32 {
    using Act = float;
    using Op = float;
    static constexpr int KL = 1;
    static constexpr bool kFP8 = false;
};
struct PBF16 {
    using Act = uint16_t;
    using Op = uint16_t;
    static constexpr int KL = 8;
    static constexpr bool kFP8 = false;
};
struct PFP8 {
    using Act = uint16_t;  // activations are stored as BF16 and quantised on load
    using Op = uint8_t;
    static constexpr int KL = 8;
    static constexpr bool kFP8 = true;
};

template <typename P>
__device__ __forceinline__ float act_to_f32(typename P::Act v) {
    if constexpr (sizeof(typename P::Act) == 4) return v;
    else return bf16_bits_to_f32(v);
}
template <typename P>
__device__ __forceinline__ typename P::Act f32_to_act(float v) {
    if constexpr (sizeof(typename P::Act) == 4) return v;
    else return f32_to_bf16_bits(v);
}

template <typename P>
__device__ __forceinline__ void mfma_step(f4v& acc, const typename P::Op* a, const typename P::Op* b) {
    if constexpr (sizeof(typename P::Op) == 4) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(*(const float*)a, *(const float*)b, acc, 0, 0, 0);
    } else if constexpr (P::kFP8) {
        long av = *(const long*)a, bv = *(const long*)b;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
    } else {
        bf16x8 av = *(const bf16x8*)a, bv = *(const bf16x8*)b;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
}

struct ConvArgs {
    const void* in;        // [B][L_in][C_in]  (P::Act)
    void* out;             // [B][L_out][C_out] (P::Act)
    const void* res;       // residual [B][L_out][C_out] or null
    const void* w;         // [C_out][KW][C_in] (P::Op)
    const float* bias;     // [C_out]
    const float* wscale;   // FP8: [C_out]
    const uint32_t* amax_in;   // FP8: [B] max |input| bit patterns
    uint32_t* amax_out;        // FP8: [B]
    int C_in, C_out, L_in, L_out, tiles_per_win;
    int relu;
};

// Implicit-GEMM conv on 16x16xMK MFMA tiles.  Workgroup = WM x WN waves; each
// wave owns TM x TN tiles.  Tile rows are output times of one window, columns
// are output channels.  K is walked in chunks of KC input channels x all taps:
// the chunk's input rows (slab) and weights are staged in LDS, then every tap
// j reads the slab shifted by j rows.
template <typename P, int KW, int S, int WM, int WN, int TM, int TN, int KC>
__global__ void __launch_bounds__(64 * WM * WN) conv_mfma_kernel(ConvArgs a) {
    using Op = typename P::Op;
    using Act = typename P::Act;
    constexpr int KL = P::KL;
    constexpr int MK = 4 * KL;
    constexpr int MT = WM * TM * 16;
    constexpr int NT = WN * TN * 16;
    constexpr int NTH = 64 * WM * WN;
    constexpr int KCH = KW * KC;                        // real k per chunk
    constexpr int KPAD = (KCH + MK - 1) / MK * MK;      // padded to whole MFMAs
    static_assert(KPAD % KC == 0, "chunk padding must be whole taps");
    static_assert(KC % KL == 0, "lane k-run must stay inside one tap");
    constexpr int KWP = KPAD / KC;                      // taps incl. zero padding
    constexpr int ROWS = (MT - 1) * S + KWP;            // slab rows
    constexpr int PA = KC + (sizeof(Op) == 4 ? 1 : 16 / (int)sizeof(Op));  // padded pitch (elements)
    constexpr int PB = PA;
    constexpr int PAD = (KW - 1) / 2;
    __shared__ __attribute__((aligned(16))) Op slab[ROWS * PA];
    __shared__ __attribute__((aligned(16))) Op wl[KWP * NT * PB];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int win = blockIdx.x / a.tiles_per_win;
    const int t0 = (blockIdx.x % a.tiles_per_win) * MT;
    const int n0 = blockIdx.y * NT;
    const Act* in = (const Act*)a.in + (size_t)win * a.L_in * a.C_in;
    const Op* wg = (const Op*)a.w;

    float inv_a = 1.f, s_a = 1.f;
    if constexpr (P::kFP8) {
        float amax = __uint_as_float(a.amax_in[win]);
        if (!(amax > 0.f)) amax = 448.f;
        inv_a = 448.f / amax;
        s_a = amax / 448.f;
    }

    f4v acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

    const int g = lane >> 4;     // lane group: k sub-range
    const int r16 = lane & 15;   // row (A) / column (B) inside a 16x16 tile

    for (int cc = 0; cc < a.C_in; cc += KC) {
        // stage the slab: rows t0*S - PAD + r, channels cc .. cc+KC
        for (int e = tid; e < ROWS * KC; e += NTH) {
            const int r = e / KC, c = e % KC;
            const int gr = t0 * S - PAD + r;
            float v = 0.f;
            if (gr >= 0 && gr < a.L_in) v = act_to_f32<P>(in[(size_t)gr * a.C_in + cc + c]);
            if constexpr (P::kFP8) slab[r * PA + c] = f32_to_e4m3(v * inv_a);
            else if constexpr (sizeof(Op) == 4) slab[r * PA + c] = v;
            else slab[r * PA + c] = f32_to_bf16_bits(v);
        }
        // stage weights: [tap][n][c] for the chunk, zero for padded taps
        for (int e = tid; e < KWP * NT * KC; e += NTH) {
            const int c = e % KC;
            const int n = (e / KC) % NT;
            const int j = e / (KC * NT);
            Op v = (Op)0;
            if (j < KW) v = wg[((size_t)(n0 + n) * KW + j) * a.C_in + cc + c];
            wl[(j * NT + n) * PB + c] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < KPAD; ks += MK) {
            const int k = ks + g * KL;
            const int j = k / KC, c = k % KC;
            const Op* ab[TM];
            const Op* bb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int row = (wm * TM + i) * 16 + r16;
                ab[i] = &slab[(row * S + j) * PA + c];
            }
#pragma unroll
            for (int jn = 0; jn < TN; ++jn) {
                const int col = (wn * TN + jn) * 16 + r16;
                bb[jn] = &wl[(j * NT + col) * PB + c];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int jn = 0; jn < TN; ++jn) mfma_step<P>(acc[i][jn], ab[i], bb[jn]);
        }
        __syncthreads();
    }

    // epilogue: dequant, bias, residual, ReLU, store, FP8 amax
    Act* out = (Act*)a.out + (size_t)win * a.L_out * a.C_out;
    const Act* res = a.res ? (const Act*)a.res + (size_t)win * a.L_out * a.C_out : nullptr;
    float vmax = 0.f;
#pragma unroll
    for (int jn = 0; jn < TN; ++jn) {
        const int col = n0 + (wn * TN + jn) * 16 + r16;
        const float bcol = a.bias[col];
        float deq = 1.f;
        if constexpr (P::kFP8) deq = s_a * a.wscale[col];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = t0 + (wm * TM + i) * 16 + g * 4 + r;
                if (t < a.L_out) {
                    float v = P::kFP8 ? fmaf(acc[i][jn][r], deq, bcol) : acc[i][jn][r] + bcol;
                    const size_t o = (size_t)t * a.C_out + col;
                    if (res) v += act_to_f32<P>(res[o]);
                    if (a.relu) v = fmaxf(v, 0.f);
                    const Act sv = f32_to_act<P>(v);
                    out[o] = sv;
                    vmax = fmaxf(vmax, fabsf(act_to_f32<P>(sv)));
                }
            }
        }
    }
    if constexpr (P::kFP8) {
        if (a.amax_out) {
            for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off));
            if (lane == 0) atomicMax(&a.amax_out[win], __float_as_uint(vmax));
        }
    }
}

struct StemArgs {
    const float* y;          // whitened series [n_ch][ld_y]
    int64_t ld_y, n, stride, wrap, first_window;
    int64_t shift[4];
    int n_ch, window;
    const float* w;          // folded stem weights [C][n_ch][KW] (FP32)
    const float* b;          // [C]
    void* out;               // [B][L_out][C] (Act)
    uint32_t* amax_out;      // FP8: [B]
    int C, KW, s0, pool, L_conv, L_out;
};

// Stem conv (vector FP32 arithmetic), ReLU, optional max-pool k3 s2 p1.
// One workgroup per window; the window's samples are staged in LDS.
template <typename P>
__global__ void __launch_bounds__(256) stem_kernel(StemArgs a) {
    using Act = typename P::Act;
    extern __shared__ float xs[];  // [n_ch][window]
    const int b = blockIdx.x;
    const int64_t wi = a.first_window + b;
    for (int e = threadIdx.x; e < a.n_ch * a.window; e += 256) {
        const int c = e / a.window, t = e % a.window;
        int64_t p = wi * a.stride + a.shift[c] + t;
        if (a.wrap > 0) p %= a.wrap;
        xs[e] = a.y[c * a.ld_y + p];
    }
    __syncthreads();
    const int pad = (a.KW - 1) / 2;
    Act* out = (Act*)a.out + (size_t)b * a.L_out * a.C;
    float vmax = 0.f;
    for (int e = threadIdx.x; e < a.L_out * a.C; e += 256) {
        const int c = e % a.C, p = e / a.C;
        const int q0 = a.pool ? 2 * p - 1 : p;
        const int q1 = a.pool ? 2 * p + 1 : p;
        float best = 0.f;  // ReLU output is >= 0, so 0 is a neutral start for the max
        for (int q = q0; q <= q1; ++q) {
            if (q < 0 || q >= a.L_conv) continue;
            float s = a.b[c];
            for (int ci = 0; ci < a.n_ch; ++ci) {
                const float* wr = a.w + ((size_t)c * a.n_ch + ci) * a.KW;
                const float* xr = xs + ci * a.window;
                for (int j = 0; j < a.KW; ++j) {
                    const int ti = q * a.s0 + j - pad;
                    if (ti >= 0 && ti < a.window) s = fmaf(wr[j], xr[ti], s);
                }
            }
            best = fmaxf(best, s);
        }
        const Act sv = f32_to_act<P>(best);
        out[e] = sv;
        vmax = fmaxf(vmax, act_to_f32<P>(sv));
    }
    if constexpr (P::kFP8) {
        for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off));
        if ((threadIdx.x & 63) == 0) atomicMax(&a.amax_out[b], __float_as_uint(vmax));
    }
}

// Global average pool over time, then FC to one logit.  One workgroup per window.
template <typename P>
__global__ void __launch_bounds__(256) gap_fc_kernel(const void* act, int L, int C, const float* fc_w,
                                                    float fc_b, float* logits) {
    using Act = typename P::Act;
    __shared__ float part[256];
    const int b = blockIdx.x;
    const Act* x = (const Act*)act + (size_t)b * L * C;
    // thread -> channel c = tid % C, time stride 256 / C (C divides 256)
    const int per = 256 / C;
    const int c = threadIdx.x % C, t0 = threadIdx.x / C;
    float s = 0.f;
    for (int t = t0; t < L; t += per) s += act_to_f32<P>(x[(size_t)t * C + c]);
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < C) {
        float tot = 0.f;
        for (int k = 0; k < per; ++k) tot += part[k * C + threadIdx.x];
        part[threadIdx.x] = tot / (float)L * fc_w[threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float z = fc_b;
        for (int k = 0; k < C; ++k) z += part[k];
        logits[b] = z;
    }
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace afm
