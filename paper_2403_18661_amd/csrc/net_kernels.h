// Device kernels of the scoring network: stem, implicit-GEMM MFMA convolution,
// global-average-pool + FC head.  Activations are stored channels-last,
// [window][time][channel], so that for a conv of kernel KW and stride S the
// implicit-GEMM row for output time t reads the contiguous input rows
// t*S - (KW-1)/2 ... t*S + (KW-1)/2 of the window.
#pragma once
#include <type_traits>
#include "common.h"

namespace afm {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));  // 16-byte staging vector
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---- scalar conversions -----------------------------------------------------
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// FP32 -> BF16 with round to nearest even: gfx950's v_cvt_pk_bf16_f32, which
// gives the bits of (u + 0x7FFF + ((u >> 16) & 1)) >> 16 for every finite
// input (checked bit for bit on the device over 2^28 patterns, ties and
// subnormals included); two values per instruction.
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2v{lo, hi}, bf16x2v));
}
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
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
// Act: stored activation element a conv reads; OAct: the one it writes (and
// its residual input); Op: LDS operand element; KL: k values per lane per
// MFMA; MK = 4 KL: k per MFMA (16x16xMK).
struct PF32 {
    using Act = float;
    using OAct = float;
    using Op = float;
    static constexpr int KL = 1;
    static constexpr bool kFP8 = false;
};
struct PBF16 {
    using Act = uint16_t;
    using OAct = uint16_t;
    using Op = uint16_t;
    static constexpr int KL = 8;
    static constexpr bool kFP8 = false;
};
struct PFP8 {
    using Act = uint16_t;  // activations are stored as BF16 and quantised on load
    using OAct = uint16_t;
    using Op = uint8_t;
    static constexpr int KL = 8;
    static constexpr bool kFP8 = true;
};
// BF16 operands with FP32 activations: every stored tensor (residual stream
// included) stays FP32 and conv operands are rounded to BF16 as they are staged
struct PBF16F {
    using Act = float;
    using OAct = float;
    using Op = uint16_t;
    static constexpr int KL = 8;
    static constexpr bool kFP8 = false;
};
// The same arithmetic with a block's inner activation stored as BF16: the
// first conv of a block reads the FP32 stream and writes its output already
// rounded the way the second conv would round it on load (PBF16FB); the
// second reads that BF16 tensor and writes the FP32 stream, adding the FP32
// skip (PBF16BF)
struct PBF16FB {
    using Act = float;
    using OAct = uint16_t;
    using Op = uint16_t;
    static constexpr int KL = 8;
    static constexpr bool kFP8 = false;
};
struct PBF16BF {
    using Act = uint16_t;
    using OAct = float;
    using Op = uint16_t;
    static constexpr int KL = 8;
    static constexpr bool kFP8 = false;
};
// FP8 on the 16x16x128 matrix instruction (32 k values per lane, unit block
// scales): twice the FP8 rate of the 16x16x32 form
struct PFP8X {
    using Act = uint16_t;
    using OAct = uint16_t;
    using Op = uint8_t;
    static constexpr int KL = 32;
    static constexpr bool kFP8 = true;
};

// GroupNorm forms of the FP32-activation traits: the conv also writes, per
// window, channel and 16-row block of its output, the sum and the sum of
// squares of the block's values (GroupNorm statistics, reduced later in a
// fixed order whatever the tile shape), and with AFF it normalises its input
// as it stages it: relu(x scale + shift) with the per-window, per-channel
// scale and shift of the previous conv's GroupNorm (zero padding stays zero).
template <typename B, bool AFF>
struct PGn : B {
    static constexpr bool kGnStats = true;
    static constexpr bool kGnAff = AFF;
};
template <typename P, typename = void>
struct GnTraits {
    static constexpr bool stats = false, aff = false;
};
template <typename P>
struct GnTraits<P, std::void_t<decltype(P::kGnStats)>> {
    static constexpr bool stats = P::kGnStats, aff = P::kGnAff;
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
    } else if constexpr (P::kFP8 && P::KL == 32) {
        typedef int i32x8 __attribute__((ext_vector_type(8)));
        // two 16-byte LDS reads per operand (rows are 16-byte aligned)
        const uint4 a0 = ((const uint4*)a)[0], a1 = ((const uint4*)a)[1];
        const uint4 b0 = ((const uint4*)b)[0], b1 = ((const uint4*)b)[1];
        const i32x8 av = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
        const i32x8 bv = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
        // formats 0/0 = E4M3 x E4M3; block scales 127 = 2^0
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc, 0, 0, 0, 127, 0, 127);
    } else if constexpr (P::kFP8) {
        long av = *(const long*)a, bv = *(const long*)b;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
    } else {
        bf16x8 av = *(const bf16x8*)a, bv = *(const bf16x8*)b;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
}

// Same product with the A operand already in registers (D dwords per lane).
template <typename P, int D>
__device__ __forceinline__ void mfma_regs(f4v& acc, const uint32_t (&a)[D], const typename P::Op* b) {
    if constexpr (P::kFP8) {
        static_assert(D == 2, "FP8 16x16x32 operands are 8 bytes per lane");
        const long av = (long)(((uint64_t)a[1] << 32) | a[0]);
        const long bv = *(const long*)b;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
    } else {
        static_assert(D == 4, "BF16 16x16x32 operands are 16 bytes per lane");
        const uint4 w = make_uint4(a[0], a[1], a[2], a[3]);
        const bf16x8 av = __builtin_bit_cast(bf16x8, w);
        const bf16x8 bv = *(const bf16x8*)b;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
}

// One lane's MFMA operand for the 16-bit and 8-bit forms, read from LDS into
// registers ahead of the product that uses it.
template <typename P>
struct Frag {
    typedef int i32x8 __attribute__((ext_vector_type(8)));
    using T = std::conditional_t<P::kFP8, std::conditional_t<P::KL == 32, i32x8, long>, bf16x8>;
};
template <typename P>
__device__ __forceinline__ typename Frag<P>::T load_frag(const typename P::Op* p) {
    using T = typename Frag<P>::T;
    if constexpr (sizeof(T) == 32) {
        const uint4 x0 = ((const uint4*)p)[0], x1 = ((const uint4*)p)[1];
        return T{(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w, (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
    } else {
        return *(const T*)p;
    }
}
template <typename P>
__device__ __forceinline__ void mfma_frag(f4v& acc, const typename Frag<P>::T& a, const typename Frag<P>::T& b) {
    if constexpr (P::kFP8 && P::KL == 32)
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
    else if constexpr (P::kFP8)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc, 0, 0, 0);
    else
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

template <int D, typename T>
__device__ __forceinline__ void load_words(uint32_t (&w)[D], const T* p) {
    if constexpr (D == 4) {
        const uint4 v = *(const uint4*)p;
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else {
        const uint2 v = *(const uint2*)p;
        w[0] = v.x; w[1] = v.y;
    }
}

struct ConvArgs {
    const void* in;        // [B][L_in][C_in]  (P::Act)
    void* out;             // [B][L_out][C_out] (P::Act)
    const void* res;       // residual [B][L_out][C_out] or null
    const void* w;         // weight image: [C_out/NT][C_in/KC][KWP][NT][PB] (P::Op), PB >= KC padded
    const float* bias;     // [C_out]
    const float* wscale;   // FP8: [C_out]
    const uint32_t* amax_in;   // FP8: [B] max |input| bit patterns
    uint32_t* amax_out;        // FP8: [B]
    int C_in, C_out, L_in, L_out;
    int n_win;             // windows in this batch
    int wpt;               // windows per M tile (tile rows = wpt x tt)
    int tt;                // output times per window per tile (multiple of 16)
    int tiles_per_win;     // M tiles per window when wpt == 1
    int relu;
    int n_mtiles;          // M tiles (set by the launcher)
    // GroupNorm forms: per window and 16-row output block, sums then sums of
    // squares over the block's rows, [B][ceil(L_out/16)][2][C_out]; and the
    // input's scale then shift, [B][2][C_in]
    float* gn_stats;
    const float* in_aff;
};

// LDS layout of the 16-byte operand reads of gfx950 (ds_read_b128 by 64
// lanes, 16 rows x 4 units of 16 bytes): rows 96 or 160 bytes apart, or
// 64-byte rows whose units are XOR-swizzled by (row / 2) & 3, are read
// without bank conflicts; 64-, 80-, 112- and 144-byte pitches and a row / 4
// swizzle conflict two ways (measured).
// Slab row pitch in elements: 32-channel 16-bit chunks get 96-byte rows,
// other chunks 16 bytes of padding.
template <int OPB, int KC>
constexpr int slab_pitch() {
    return (OPB == 2 && KC == 32) ? KC + 16 : KC + 16 / OPB;
}
// Rows per step of the XOR swizzle of unpadded 16/8-bit weight rows (0: the
// FP32 rows are padded instead).
template <int OPB, int KC>
constexpr int weight_swizzle_rows() {
    if constexpr (OPB == 4) return 0;
    else if constexpr (OPB == 2 && KC == 32) return 2;
    else return 256 / (KC * OPB) > 0 ? 256 / (KC * OPB) : 1;
}

template <int KW, int KC, int MK>
struct ChunkGeom {
    static constexpr int KCH = KW * KC;
    static constexpr int KPAD = (KCH + MK - 1) / MK * MK;
    static constexpr int KWP = KPAD / KC;
};

// Two packed BF16 words (4 values) -> 4 E4M3 bytes after scaling by sc.
// gfx950's packed FP32 -> OCP E4M3 conversion rounds to nearest even like
// f32_to_e4m3 (checked bit for bit on the device for |x| <= 448); the clamp
// keeps it on the saturating side where it would otherwise return NaN.
__device__ __forceinline__ uint32_t pack_e4m3x4(uint32_t lo2, uint32_t hi2, float sc) {
    auto q = [](float v) { return fminf(fmaxf(v, -448.f), 448.f); };
    const float a = q(__uint_as_float(lo2 << 16) * sc), b = q(__uint_as_float(lo2 & 0xFFFF0000u) * sc);
    const float c = q(__uint_as_float(hi2 << 16) * sc), d = q(__uint_as_float(hi2 & 0xFFFF0000u) * sc);
    int r = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    r = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, r, true);
    return (uint32_t)r;
}

// Implicit-GEMM conv on 16x16xMK MFMA tiles.
// Workgroup = WM x WN waves, each wave TM x TN tiles of 16x16 outputs.  The M
// tile covers `wpt` windows x `tt` output times; the N tile NT output channels.
// K is walked in chunks of KC input channels x all KW taps.  Per chunk the
// input rows of every window in the tile (the slab, rows t*S - (KW-1)/2 ...)
// and the chunk's weights are staged in LDS with 16-byte loads; tap j then
// reads the slab shifted by j rows.  Staging (DB): 0, one LDS buffer, each
// chunk fetched and stored between two barriers; 1, two LDS buffers, the next
// chunk fetched into registers while the current one is multiplied and
// stored into the other buffer; 2, one LDS buffer, the next chunk fetched
// into registers during the MFMAs and stored between two barriers.
// Waves per SIMD the register allocation aims for: three for the small
// 16/8-bit tiles with 16- or 8-byte operands in one LDS buffer (whose LDS
// lets three workgroups share a CU), two when such a tile holds the next
// chunk's FP32 activations in registers (three would spill); four for the
// eight-wave 16/8-bit tiles in one buffer (two workgroups per CU);
// otherwise the compiler's choice.
template <typename P, int WM, int WN, int TM, int TN, int DB>
constexpr int conv_waves_per_eu() {
    if constexpr (DB == 0 && WM * WN == 8 && sizeof(typename P::Op) <= 2 && P::KL <= 8)
        return 4;
    else if constexpr (DB != 1 && sizeof(typename P::Op) <= 2 && P::KL <= 8 && WM * TM * WN * TN * 256 <= 192 * 64)
        return (DB == 2 && sizeof(typename P::Act) == 4) ? 2 : 3;
    else
        return 1;
}

template <typename P, int KW, int S, int WM, int WN, int TM, int TN, int KC, int WMAX, int DB, bool TS = true>
__global__ void __launch_bounds__(64 * WM * WN, (conv_waves_per_eu<P, WM, WN, TM, TN, DB>()))
    conv_mfma_kernel(ConvArgs a) {
    using Op = typename P::Op;
    using Act = typename P::Act;
    using OAct = typename P::OAct;
    constexpr int KL = P::KL;
    constexpr int MK = 4 * KL;
    constexpr int MT = WM * TM * 16;
    constexpr int NT = WN * TN * 16;
    constexpr int NTH = 64 * WM * WN;
    using G = ChunkGeom<KW, KC, MK>;
    constexpr int KPAD = G::KPAD, KWP = G::KWP;
    static_assert(KPAD % KC == 0, "chunk padding must be whole taps");
    static_assert(KC % KL == 0, "lane k-run must stay inside one tap");
    constexpr int OPB = (int)sizeof(Op);
    constexpr int PA = slab_pitch<OPB, KC>();   // slab row pitch in elements
    // weight row pitch: FP32 lanes read 4 B (pad 4); 32-byte FP8 lane reads (pad 16 B)
    constexpr int PB = OPB == 4 ? KC + 4 : (KL == 32 ? KC + 16 : KC);
    // BF16/FP8 weight rows are not padded; instead the KL-element units of row
    // r are XOR-swizzled by (r / SWR) & (KC/KL - 1), so that the 16 rows one
    // MFMA operand read touches fall in distinct LDS banks
    constexpr int SWU = KC / KL;                                    // units per row
    constexpr int SWR = weight_swizzle_rows<OPB, KC>();
    // tap-shift reuse of the A operand (see the k-loop)
    constexpr bool SHIFT = TS && S == 1 && KW > 1 && MK == KC && KPAD == KW * KC && OPB <= 2 && KL == 8;
    constexpr int PAD = (KW - 1) / 2;
    // rows of all windows' slabs: wpt windows need (MT - wpt) S + wpt KWP rows,
    // largest at wpt = WMAX when KWP >= S and at wpt = 1 otherwise (1x1, stride 2)
    constexpr int ROWS_W1 = (MT - 1) * S + KWP;
    constexpr int ROWS_WMAX = (MT - WMAX) * S + WMAX * KWP;
    constexpr int SLAB_ROWS = ROWS_W1 > ROWS_WMAX ? ROWS_W1 : ROWS_WMAX;
    constexpr int SLAB_EL = SLAB_ROWS * PA;
    constexpr int W_EL = KWP * NT * PB;
    static_assert(DB >= 0 && DB <= 2, "staging mode");
    constexpr bool LDS2 = DB == 1;   // two LDS buffers
    constexpr bool PREF = DB != 0;   // next chunk fetched into registers during the MFMAs
    constexpr int NBUF = LDS2 ? 2 : 1;
    // slab: 16-byte vectors through registers.  Weights (the chunk's LDS image,
    // padding included): with PREF also through registers, loaded at the
    // start of the chunk before and written to LDS at its end, since a direct
    // global->LDS copy in flight makes every LDS read of the current chunk
    // wait for it (the wait counters cannot tell the buffers apart); without
    // PREF nothing overlaps, and direct global->LDS copies save the registers
    constexpr int AE = 16 / (int)sizeof(Act);   // activations per 16-byte load
    constexpr int AV_ROW = KC / AE;             // vectors per slab row
    static_assert(KC % AE == 0, "slab rows must be whole 16-byte vectors");
    constexpr int AV_MAX = SLAB_ROWS * AV_ROW;
    constexpr int RA = (AV_MAX + NTH - 1) / NTH;  // slab vectors per thread (upper bound)
    constexpr int W_BYTES = W_EL * OPB;           // one chunk's weight image
    static_assert(W_BYTES % 16 == 0 && (SLAB_EL * OPB) % 16 == 0, "16-byte LDS regions");
    constexpr int WV = W_BYTES / 16;              // 16-byte vectors of the weight image
    constexpr int RW = PREF ? (WV + NTH - 1) / NTH : 1;  // weight vectors per thread (PREF)
    constexpr int W_INST = (W_BYTES + 1023) / 1024;      // wave-wide 1 KB copies (no PREF)
    constexpr int NWAVES = WM * WN;
    // the epilogue reuses the same LDS for the FP32 output tile [MT][NT + 4],
    // in EPH row phases of MTP rows: tall tiles of waves stacked along M
    // stage half of their rows at a time so that the epilogue does not need
    // more LDS than the main loop
    constexpr int EPITCH = NT + 4;
    constexpr int EPH = (WN == 1 && WM % 2 == 0 && MT >= 384) ? 2 : 1;
    constexpr int MTP = MT / EPH;
    constexpr int BUF_BYTES = NBUF * (SLAB_EL + W_EL) * OPB;
    constexpr int EPI_BYTES = MTP * EPITCH * 4;
    constexpr int SMEM_BYTES = BUF_BYTES > EPI_BYTES ? BUF_BYTES : EPI_BYTES;
    __shared__ __attribute__((aligned(16))) unsigned char smem_raw[SMEM_BYTES];
    Op* smem = (Op*)smem_raw;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int g = lane >> 4;     // lane group: k sub-range
    const int r16 = lane & 15;   // row (A) / column (B) inside a 16x16 tile
    const int wpt = a.wpt, tt = a.tt;
    const int srows = (tt - 1) * S + KWP;   // slab rows per window
    // Workgroup order: consecutive workgroups go to the 8 XCDs in turn.  Each
    // XCD takes a contiguous range of M tiles and, for each, all N tiles one
    // after another, so that the N tiles reading one input slab run together
    // and find it in that XCD's L2.  The grid is rounded up to whole ranges;
    // the surplus workgroups return at once.
    const int n_nt = a.C_out / NT;
    const int per_xcd = (a.n_mtiles + 7) >> 3;
    const int kx = (int)(blockIdx.x >> 3);
    const int mtile = (int)(blockIdx.x & 7) * per_xcd + kx / n_nt;
    const int nt = kx % n_nt;
    if (mtile >= a.n_mtiles) return;
    int win0, t0;
    if (wpt == 1) {
        win0 = mtile / a.tiles_per_win;
        t0 = (mtile % a.tiles_per_win) * tt;
    } else {
        win0 = mtile * wpt;
        t0 = 0;
    }
    const int n0 = nt * NT;
    const int n_chunks = a.C_in / KC;
    const Act* in = (const Act*)a.in;
    const char* wimg = (const char*)a.w + (size_t)nt * n_chunks * W_BYTES;

    // FP8: per-window activation scales of the windows in this tile
    float inv_a[WMAX], s_a[WMAX];
#pragma unroll
    for (int w = 0; w < WMAX; ++w) {
        inv_a[w] = 1.f;
        s_a[w] = 1.f;
        if constexpr (P::kFP8) {
            if (w < wpt && win0 + w < a.n_win) {
                float amax = __uint_as_float(a.amax_in[win0 + w]);
                if (!(amax > 0.f)) amax = 448.f;
                inv_a[w] = 448.f / amax;
                s_a[w] = amax / 448.f;
            }
        }
    }

    const int av_count = wpt * srows * AV_ROW;
    uint4 ra[RA];
    f4v acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

    // slab row offsets of this lane's A rows (window-relative layout)
    int arow[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int row = (wm * TM + i) * 16 + r16;
        const int w = row / tt, t = row % tt;
        arow[i] = (w * srows + t * S) * PA;
    }

    // slab vectors of this thread: source offset from the tile's first window
    // (without the chunk's channel offset), LDS offset, validity and (FP8)
    // scale, all chunk-independent
    const Act* in_t = in + (size_t)win0 * a.L_in * a.C_in;
    int f_off[RA];
    int s_off[RA];
    bool f_ok[RA], s_ok[RA];
    float s_sc[RA];
    int f_w[RA];   // window of the vector within the tile (GroupNorm input scaling)
#pragma unroll
    for (int i = 0; i < RA; ++i) {
        const int v = tid + i * NTH;
        const int q = v % AV_ROW;
        const int rr = v / AV_ROW;
        const int w = rr / srows, r = rr % srows;
        const int gr = t0 * S - PAD + r;
        const int win = win0 + w;
        s_ok[i] = v < av_count;
        f_ok[i] = s_ok[i] && win < a.n_win && gr >= 0 && gr < a.L_in;
        f_off[i] = f_ok[i] ? (w * a.L_in + gr) * a.C_in + q * AE : 0;
        s_off[i] = rr * PA + q * AE;
        f_w[i] = w;
        float sc = inv_a[0];
#pragma unroll
        for (int u = 1; u < WMAX; ++u) sc = (w == u) ? inv_a[u] : sc;
        s_sc[i] = sc;
    }
    // GroupNorm input scaling: a thread's vectors all start at channel
    // q * AE of the chunk (NTH is a multiple of AV_ROW), so per chunk it needs
    // one scale and one shift vector per window of the tile
    constexpr bool GAFF = GnTraits<P>::aff;
    static_assert(!GAFF || (sizeof(Act) == 4 && NTH % AV_ROW == 0), "GroupNorm input scaling reads FP32 rows");
    const int q_t = tid % AV_ROW;
    float4 gsc[GAFF ? WMAX : 1] = {}, gsh[GAFF ? WMAX : 1] = {};
#define AFM_FETCH(CC)                                                                              \
    {                                                                                              \
        _Pragma("unroll") for (int i = 0; i < RA; ++i) {                                          \
            uint4 x = make_uint4(0u, 0u, 0u, 0u);                                                  \
            if (f_ok[i]) x = *(const uint4*)(in_t + f_off[i] + (CC) * KC);                         \
            ra[i] = x;                                                                             \
        }                                                                                          \
        if constexpr (GAFF) {                                                                      \
            _Pragma("unroll") for (int u = 0; u < WMAX; ++u) {                                    \
                if (u == 0 || u < wpt) {                                                           \
                    const int wu = win0 + u;                                                       \
                    const float* ap_ = a.in_aff + (size_t)(wu < a.n_win ? wu : a.n_win - 1) * 2 * a.C_in \
                                       + (CC) * KC + q_t * AE;                                     \
                    gsc[u] = *(const float4*)ap_;                                                  \
                    gsh[u] = *(const float4*)(ap_ + a.C_in);                                       \
                }                                                                                  \
            }                                                                                      \
        }                                                                                          \
    }
#define AFM_WLOAD(RWV, CC, BUF)                                                                    \
    if constexpr (PREF) {                                                                          \
        const uint4* src_ = (const uint4*)(wimg + (size_t)(CC) * W_BYTES);                        \
        _Pragma("unroll") for (int i = 0; i < RW; ++i) {                                          \
            const int u = tid + i * NTH;                                                           \
            if (WV % NTH == 0 || u < WV) RWV[i] = *(const u4v*)(src_ + u);                        \
        }                                                                                          \
    } else {                                                                                       \
        const char* src_ = wimg + (size_t)(CC) * W_BYTES;                                          \
        char* dst_ = (char*)(smem + (BUF) * (SLAB_EL + W_EL) + SLAB_EL);                           \
        for (int i = wave; i < W_INST; i += NWAVES) {                                              \
            const int o = i * 1024 + lane * 16;                                                    \
            if (W_BYTES % 1024 == 0 || o < W_BYTES)                                                \
                __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(src_ + o), \
                                                 (__attribute__((address_space(3))) void*)(dst_ + i * 1024), 16, 0, 0); \
        }                                                                                          \
    }
#define AFM_STASH(RWV, BUF)                                                                        \
    {                                                                                              \
        Op* slab_ = smem + (BUF) * (SLAB_EL + W_EL);                                               \
        if constexpr (PREF) {                                                                      \
            uint4* wdst_ = (uint4*)(slab_ + SLAB_EL);                                              \
            _Pragma("unroll") for (int i = 0; i < RW; ++i) {                                      \
                const int u = tid + i * NTH;                                                       \
                if (WV % NTH == 0 || u < WV) *(u4v*)(wdst_ + u) = RWV[i];                          \
            }                                                                                      \
        }                                                                                          \
        _Pragma("unroll") for (int i = 0; i < RA; ++i) {                                          \
            if (s_ok[i]) {                                                                         \
                Op* dst = slab_ + s_off[i];                                                        \
                if constexpr (GAFF) {                                                              \
                    float4 sc_ = gsc[0], sh_ = gsh[0];                                             \
                    if (wpt > 1) {   /* several windows per tile (uniform) */                      \
                        _Pragma("unroll") for (int u = 1; u < WMAX; ++u)                          \
                            if (f_w[i] == u) { sc_ = gsc[u]; sh_ = gsh[u]; }                       \
                    }                                                                              \
                    if (f_ok[i])                                                                   \
                        ra[i] = make_uint4(                                                        \
                            __float_as_uint(fmaxf(fmaf(__uint_as_float(ra[i].x), sc_.x, sh_.x), 0.f)), \
                            __float_as_uint(fmaxf(fmaf(__uint_as_float(ra[i].y), sc_.y, sh_.y), 0.f)), \
                            __float_as_uint(fmaxf(fmaf(__uint_as_float(ra[i].z), sc_.z, sh_.z), 0.f)), \
                            __float_as_uint(fmaxf(fmaf(__uint_as_float(ra[i].w), sc_.w, sh_.w), 0.f))); \
                }                                                                                  \
                if constexpr (sizeof(Act) == 4 && sizeof(Op) == 2) {                               \
                    const uint4 f = ra[i];                                                         \
                    *(uint2*)dst = make_uint2(pack_bf16x2(__uint_as_float(f.x), __uint_as_float(f.y)),  \
                                              pack_bf16x2(__uint_as_float(f.z), __uint_as_float(f.w))); \
                } else if constexpr (P::kFP8) {                                                    \
                    const float sc = s_sc[i];                                                      \
                    *(uint2*)dst = make_uint2(pack_e4m3x4(ra[i].x, ra[i].y, sc),                    \
                                              pack_e4m3x4(ra[i].z, ra[i].w, sc));                   \
                } else {                                                                           \
                    *(uint4*)dst = ra[i];                                                          \
                }                                                                                  \
            }                                                                                      \
        }                                                                                          \
    }

    {
        u4v rw[RW];
        AFM_FETCH(0)
        AFM_WLOAD(rw, 0, 0)
        AFM_STASH(rw, 0)
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int cc = 0; cc < n_chunks; ++cc) {
        const int buf = LDS2 ? (cc & 1) : 0;
        u4v rw[RW];  // the next chunk's weights (PREF), loaded now, stored to LDS after the MFMAs
        if (PREF && cc + 1 < n_chunks) {
            AFM_FETCH(cc + 1)
            AFM_WLOAD(rw, cc + 1, buf ^ 1)
        }
        const Op* slab = smem + buf * (SLAB_EL + W_EL);
        const Op* wl = slab + SLAB_EL;
        if constexpr (SHIFT) {
            // stride 1, one tap per k-step: the A operand of tap j+1 is the one
            // of tap j moved up one row.  Rotate it left by one lane within each
            // 16-lane row (DPP row_ror:15) and let lane 15 of every row read
            // the one new slab row from LDS (4 active lanes per tile).
            constexpr int D = KL * OPB / 4;
            uint32_t af[TM][D];
#pragma unroll
            for (int i = 0; i < TM; ++i) load_words<D>(af[i], slab + arow[i] + g * KL);
#pragma unroll
            for (int j = 0; j < KW; ++j) {
                const int c = g * KL;
                const Op* bb[TN];
#pragma unroll
                for (int jn = 0; jn < TN; ++jn) {
                    const int row = j * NT + (wn * TN + jn) * 16 + r16;
                    const int cs = SWR ? (((c / KL) ^ ((row / (SWR ? SWR : 1)) & (SWU - 1))) * KL) : c;
                    bb[jn] = wl + row * PB + cs;
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int jn = 0; jn < TN; ++jn) mfma_regs<P, D>(acc[i][jn], af[i], bb[jn]);
                if (j + 1 < KW) {
#pragma unroll
                    for (int i = 0; i < TM; ++i) {
                        uint32_t ex[D];
#pragma unroll
                        for (int d = 0; d < D; ++d) ex[d] = 0u;
                        if (r16 == 15) load_words<D>(ex, slab + arow[i] + (j + 1) * PA + g * KL);
#pragma unroll
                        for (int d = 0; d < D; ++d) {
                            const uint32_t rot = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)af[i][d], 0x12F, 0xF, 0xF, false);
                            af[i][d] = r16 == 15 ? ex[d] : rot;
                        }
                    }
                }
            }
        } else if constexpr (OPB <= 2) {
            // two-stage register pipeline: the fragments of k-step s + 1 are
            // read from LDS before the MFMAs of step s are issued
            using FT = typename Frag<P>::T;
            constexpr int NS = KPAD / MK;
            FT fa[2][TM], fb[2][TN];
            auto load_step = [&](int ks, FT (&xa)[TM], FT (&xb)[TN]) {
                const int k = ks * MK + g * KL;
                const int j = k / KC, c = k % KC;
#pragma unroll
                for (int i = 0; i < TM; ++i) xa[i] = load_frag<P>(slab + arow[i] + j * PA + c);
#pragma unroll
                for (int jn = 0; jn < TN; ++jn) {
                    const int row = j * NT + (wn * TN + jn) * 16 + r16;
                    const int cs = SWR ? (((c / KL) ^ ((row / (SWR ? SWR : 1)) & (SWU - 1))) * KL) : c;
                    xb[jn] = load_frag<P>(wl + row * PB + cs);
                }
            };
            load_step(0, fa[0], fb[0]);
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                if (st + 1 < NS) load_step(st + 1, fa[(st + 1) & 1], fb[(st + 1) & 1]);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int jn = 0; jn < TN; ++jn) mfma_frag<P>(acc[i][jn], fa[st & 1][i], fb[st & 1][jn]);
            }
        } else
#pragma unroll
        for (int ks = 0; ks < KPAD; ks += MK) {
            const int k = ks + g * KL;
            const int j = k / KC, c = k % KC;
            const Op* ab[TM];
            const Op* bb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) ab[i] = slab + arow[i] + j * PA + c;
#pragma unroll
            for (int jn = 0; jn < TN; ++jn) {
                const int row = j * NT + (wn * TN + jn) * 16 + r16;
                const int cs = SWR ? (((c / KL) ^ ((row / (SWR ? SWR : 1)) & (SWU - 1))) * KL) : c;
                bb[jn] = wl + row * PB + cs;
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int jn = 0; jn < TN; ++jn) mfma_step<P>(acc[i][jn], ab[i], bb[jn]);
        }
        if (LDS2) {
            if (cc + 1 < n_chunks) AFM_STASH(rw, buf ^ 1)
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        } else if (PREF) {
            if (cc + 1 < n_chunks) {
                __syncthreads();   // every wave is done reading this chunk
                AFM_STASH(rw, 0)
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
            }
        } else if (cc + 1 < n_chunks) {
            __syncthreads();
            AFM_FETCH(cc + 1)
            AFM_WLOAD(rw, cc + 1, 0)
            AFM_STASH(rw, 0)
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
    }
#undef AFM_FETCH
#undef AFM_WLOAD
#undef AFM_STASH

    if constexpr (GnTraits<P>::stats) {
        // GroupNorm statistics, straight from the accumulators: tile i of a
        // wave is one 16-row block of the output (tt and t0 are multiples of
        // 16, so the block lies in one window and starts at a multiple of
        // 16), whose column r16 this lane holds at rows 4g .. 4g + 3.  These
        // convs have no bias, residual or ReLU, so the accumulators are the
        // values stored.  They are summed in the lane in row order, then
        // across the lane groups (xor 16, then xor 32): the same order
        // whatever the tile shape.
        const int nblk = (a.L_out + 15) >> 4;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int row0 = (wm * TM + i) * 16;
            const int w = row0 / tt, tb = t0 + row0 % tt;
            const bool ok = win0 + w < a.n_win && tb < a.L_out;
            const int nval = a.L_out - tb;   // rows of the block inside the output (> 16: all)
#pragma unroll
            for (int jn = 0; jn < TN; ++jn) {
                const int col = (wn * TN + jn) * 16 + r16;
                float sum = 0.f, sq = 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (g * 4 + r < nval) {
                        const float x = acc[i][jn][r];
                        sum += x;
                        sq = fmaf(x, x, sq);
                    }
                }
                sum += __shfl_xor(sum, 16);
                sq += __shfl_xor(sq, 16);
                sum += __shfl_xor(sum, 32);
                sq += __shfl_xor(sq, 32);
                if (ok && g == 0) {
                    float* st = a.gn_stats + ((size_t)(win0 + w) * nblk + (tb >> 4)) * 2 * a.C_out + n0 + col;
                    st[0] = sum;
                    st[a.C_out] = sq;
                }
            }
        }
    }

    // epilogue: the accumulators go through LDS so that bias, dequant,
    // residual, ReLU, rounding and the stores run on 16-byte row vectors
    float* et = (float*)smem_raw;
    constexpr int VE = 16 / (int)sizeof(OAct);   // outputs per 16-byte vector
    constexpr int VPR = NT / VE;                // vectors per tile row
    constexpr int EPI_IT = (MTP * VPR + NTH - 1) / NTH;
    float vmax[WMAX];
#pragma unroll
    for (int u = 0; u < WMAX; ++u) vmax[u] = 0.f;
    // NTH is a multiple of VPR, so a thread's columns are the same in every
    // iteration: its bias (and FP8 weight scales) are loaded once
    static_assert(NTH % VPR == 0, "epilogue columns must not depend on the iteration");
    const int col_t = (tid % VPR) * VE;
    float bcol[VE], scol[VE];
#pragma unroll
    for (int e = 0; e < VE; ++e) {
        bcol[e] = a.bias[n0 + col_t + e];
        scol[e] = P::kFP8 ? a.wscale[n0 + col_t + e] : 1.f;
    }
#pragma unroll
    for (int ph = 0; ph < EPH; ++ph) {
    __syncthreads();
    if (EPH == 1 || wm / (WM / EPH) == ph) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int jn = 0; jn < TN; ++jn)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    et[((wm * TM + i) * 16 + g * 4 + r - ph * MTP) * EPITCH + (wn * TN + jn) * 16 + r16] = acc[i][jn][r];
    }
    __syncthreads();
    // all residual loads first (a thread reads and later writes the same
    // elements, so this also holds when the output overwrites the residual)
    uint4 rres[EPI_IT];
    size_t ooff[EPI_IT];
    bool oval[EPI_IT];
#pragma unroll
    for (int it = 0; it < EPI_IT; ++it) {
        const int v = tid + it * NTH;
        const int row = ph * MTP + v / VPR, col = (v % VPR) * VE;
        const int w = row / tt;
        const int t = t0 + row % tt;
        oval[it] = v < MTP * VPR && win0 + w < a.n_win && t < a.L_out;
        ooff[it] = ((size_t)(win0 + w) * a.L_out + t) * a.C_out + n0 + col;
        rres[it] = make_uint4(0u, 0u, 0u, 0u);
        if (a.res && oval[it]) rres[it] = *(const uint4*)((const OAct*)a.res + ooff[it]);
    }
    // BF16/FP8 operands: every tile row read from LDS first (rows < MT: always
    // in range), so the reads of all iterations are in flight together and
    // only stores are guarded.  FP32 reads per iteration instead: the extra
    // registers would cost its kernels a wave per SIMD.
    constexpr bool XPRE = OPB <= 2;
    float xt[XPRE ? EPI_IT : 1][VE];
    if constexpr (XPRE) {
#pragma unroll
        for (int it = 0; it < EPI_IT; ++it) {
            const int v = tid + it * NTH;
            const int lrow = (v < MTP * VPR ? v : 0) / VPR;
#pragma unroll
            for (int e = 0; e < VE; ++e) xt[it][e] = et[lrow * EPITCH + col_t + e];
        }
    }
#pragma unroll
    for (int it = 0; it < EPI_IT; ++it) {
        if (!oval[it]) continue;
        const int v = tid + it * NTH;
        const int lrow = v / VPR;
        const int w = (ph * MTP + lrow) / tt;
        float x[VE];
#pragma unroll
        for (int e = 0; e < VE; ++e) x[e] = XPRE ? xt[XPRE ? it : 0][e] : et[lrow * EPITCH + col_t + e];
        float sa = 1.f;
        if constexpr (P::kFP8) {
            sa = s_a[0];
#pragma unroll
            for (int u = 1; u < WMAX; ++u) sa = (w == u) ? s_a[u] : sa;
        }
#pragma unroll
        for (int e = 0; e < VE; ++e) x[e] = P::kFP8 ? fmaf(x[e], sa * scol[e], bcol[e]) : x[e] + bcol[e];
        if (a.res) {
            const uint4 rv = rres[it];
            if constexpr (sizeof(OAct) == 4) {
                x[0] += __uint_as_float(rv.x); x[1] += __uint_as_float(rv.y);
                x[2] += __uint_as_float(rv.z); x[3] += __uint_as_float(rv.w);
            } else {
                const uint32_t wv[4] = {rv.x, rv.y, rv.z, rv.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    x[2 * e] += __uint_as_float(wv[e] << 16);
                    x[2 * e + 1] += __uint_as_float(wv[e] & 0xFFFF0000u);
                }
            }
        }
        if (a.relu) {
#pragma unroll
            for (int e = 0; e < VE; ++e) x[e] = fmaxf(x[e], 0.f);
        }
        uint4 ov;
        float m = 0.f;
        if constexpr (sizeof(OAct) == 4) {
            ov = make_uint4(__float_as_uint(x[0]), __float_as_uint(x[1]), __float_as_uint(x[2]), __float_as_uint(x[3]));
            m = fmaxf(fmaxf(fabsf(x[0]), fabsf(x[1])), fmaxf(fabsf(x[2]), fabsf(x[3])));
        } else {
            uint32_t wv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                wv[e] = pack_bf16x2(x[2 * e], x[2 * e + 1]);
                if constexpr (P::kFP8)
                    m = fmaxf(m, fmaxf(fabsf(__uint_as_float(wv[e] << 16)), fabsf(__uint_as_float(wv[e] & 0xFFFF0000u))));
            }
            ov = make_uint4(wv[0], wv[1], wv[2], wv[3]);
        }
        *(uint4*)((OAct*)a.out + ooff[it]) = ov;
        if constexpr (P::kFP8) {
#pragma unroll
            for (int u = 0; u < WMAX; ++u)
                if (w == u) vmax[u] = fmaxf(vmax[u], m);
        }
    }
    }   // epilogue phases
    if constexpr (P::kFP8) {
        if (a.amax_out) {
#pragma unroll
            for (int u = 0; u < WMAX; ++u) {
                float vm = vmax[u];
                for (int off = 32; off > 0; off >>= 1) vm = fmaxf(vm, __shfl_xor(vm, off));
                if (lane == 0 && u < wpt && win0 + u < a.n_win) atomicMax(&a.amax_out[win0 + u], __float_as_uint(vm));
            }
        }
    }
}

struct StemArgs {
    const float* y;          // whitened series [n_ch][ld_y]
    int64_t ld_y, n, stride, wrap, first_window;
    int64_t shift[4];
    // timeslide work table (device): per entry {segment offset, segment length,
    // shift of channels >= 1, first global window}; null for plain windows
    const int64_t* table;
    int n_entries;
    int n_ch, window;
    const float* w;          // folded stem weights [C][n_ch][KW] (FP32)
    const float* b;          // [C]
    void* out;               // [B][L_out][C] (Act)
    uint32_t* amax_out;      // FP8: [B]
    int C, KW, s0, pool, L_conv, L_out;
};

// Where window `wi` reads channel c: sample (start[c] + t) mod wrap (no mod
// when wrap == 0) of y[c] + base.  Plain mode: start = wi*stride + shift[c].
// Timeslide mode: the entry holding wi gives a segment [base, base + len);
// channel 0 starts at i*stride and the others at i*stride + shift, both
// circular within the segment.
struct WinAddr {
    int64_t base, wrap;
    int64_t start[4];
};

__device__ __forceinline__ WinAddr window_addr(const StemArgs& a, int64_t wi) {
    WinAddr w;
    if (a.table) {
        int lo = 0, hi = a.n_entries - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.table[4 * mid + 3] <= wi) lo = mid; else hi = mid - 1;
        }
        const int64_t* e = a.table + 4 * lo;
        const int64_t i0 = (wi - e[3]) * a.stride;
        w.base = e[0];
        w.wrap = e[1];
        for (int c = 0; c < 4; ++c) w.start[c] = c == 0 ? i0 : i0 + e[2];
    } else {
        w.base = 0;
        w.wrap = a.wrap;
        for (int c = 0; c < 4; ++c) w.start[c] = wi * a.stride + a.shift[c];
    }
    // starts are non-negative; reduced here once, so that with t < window <=
    // wrap a sample index passes the end at most once
    if (w.wrap > 0)
        for (int c = 0; c < 4; ++c) w.start[c] %= w.wrap;
    return w;
}

__device__ __forceinline__ int64_t window_sample(const WinAddr& w, int c, int t) {
    // select, not an indexed load: a run-time index would put start[] in scratch
    const int64_t st = c == 0 ? w.start[0] : c == 1 ? w.start[1] : c == 2 ? w.start[2] : w.start[3];
    const int64_t p = st + t;
    return w.base + ((w.wrap > 0 && p >= w.wrap) ? p - w.wrap : p);
}

// Stage a window's samples, [n_ch][window] floats (n_ch <= 4), into LDS with
// 256 threads, channel c at xs[c * pitch + padl + t] (pitch 0: the window
// length).  Each thread issues up to SB loads before it stores any, so that
// their latencies overlap (a load-then-store loop waits on every load); loads
// past the end read a clamped, valid index and are not stored.
__device__ __forceinline__ void stage_window(const StemArgs& a, const WinAddr& wa, float* xs, int pitch = 0,
                                             int padl = 0) {
    constexpr int SB = 12;
    const int W = a.window;
    const int pw = pitch ? pitch : W;
    for (int c = 0; c < a.n_ch; ++c) {
        const float* yc = a.y + c * a.ld_y + wa.base;
        const int64_t st = c == 0 ? wa.start[0] : c == 1 ? wa.start[1] : c == 2 ? wa.start[2] : wa.start[3];
        for (int t0 = threadIdx.x; t0 < W; t0 += 256 * SB) {
            float v[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int64_t p = st + min(t0 + u * 256, W - 1);
                v[u] = yc[(wa.wrap > 0 && p >= wa.wrap) ? p - wa.wrap : p];
            }
#pragma unroll
            for (int u = 0; u < SB; ++u)
                if (t0 + u * 256 < W) xs[c * pw + padl + t0 + u * 256] = v[u];
        }
    }
}

// Stem conv (vector FP32 arithmetic), ReLU, optional max-pool k3 s2 p1.
// One workgroup per window; the window's samples are staged in LDS.
template <typename P>
__global__ void __launch_bounds__(256) stem_kernel(StemArgs a) {
    using Act = typename P::Act;
    extern __shared__ float xs[];  // [n_ch][window]
    const int b = blockIdx.x;
    const int64_t wi = a.first_window + b;
    const WinAddr wa = window_addr(a, wi);
    stage_window(a, wa, xs);
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

// Stem for two detectors and kernel 7, one thread per output time with all C
// channels in registers; weights are uniform across the workgroup (scalar
// loads).  With POOL each thread evaluates the three conv outputs 2p-1..2p+1
// under its max-pool window.  One workgroup per window, samples staged in LDS.
template <typename P, int C, int S0, bool POOL>
__global__ void __launch_bounds__(256) stem2_kernel(StemArgs a) {
    using Act = typename P::Act;
    constexpr int KW = 7, PADS = 3, NCH = 2;
    constexpr int QN = POOL ? 3 : 1;
    constexpr int NIN = (QN - 1) * S0 + KW;   // input samples per channel per thread
    extern __shared__ float xs[];             // [NCH][window]
    const int b = blockIdx.x;
    const int64_t wi = a.first_window + b;
    const int W = a.window;
    const WinAddr wa = window_addr(a, wi);
    stage_window(a, wa, xs);   // a.n_ch == NCH
    __syncthreads();
    Act* out = (Act*)a.out + (size_t)b * a.L_out * C;
    const float* __restrict__ wt = a.w;   // [C][NCH][KW]
    const float* __restrict__ bs = a.b;
    float vmax = 0.f;
    for (int p = threadIdx.x; p < a.L_out; p += 256) {
        const int q0 = POOL ? 2 * p - 1 : p;
        const int i0 = q0 * S0 - PADS;        // first input sample
        float xin[NCH][NIN];
#pragma unroll
        for (int ci = 0; ci < NCH; ++ci)
#pragma unroll
            for (int u = 0; u < NIN; ++u) {
                const int ti = i0 + u;
                xin[ci][u] = (ti >= 0 && ti < W) ? xs[ci * W + ti] : 0.f;
            }
        float res[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float best = 0.f;   // ReLU output >= 0; an out-of-range pool position never wins
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                float sacc = bs[c];
#pragma unroll
                for (int ci = 0; ci < NCH; ++ci)
#pragma unroll
                    for (int j = 0; j < KW; ++j) sacc = fmaf(wt[(c * NCH + ci) * KW + j], xin[ci][q * S0 + j], sacc);
                const int qq = q0 + q;
                if (!POOL || (qq >= 0 && qq < a.L_conv)) best = fmaxf(best, sacc);
            }
            res[c] = best;
        }
        Act* o = out + (size_t)p * C;
        if constexpr (sizeof(Act) == 4) {
#pragma unroll
            for (int c = 0; c < C; c += 4) {
                *(float4*)(o + c) = make_float4(res[c], res[c + 1], res[c + 2], res[c + 3]);
                vmax = fmaxf(vmax, fmaxf(fmaxf(res[c], res[c + 1]), fmaxf(res[c + 2], res[c + 3])));
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; c += 8) {
                uint32_t u4[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    u4[e] = pack_bf16x2(res[c + 2 * e], res[c + 2 * e + 1]);
                    if constexpr (P::kFP8)
                        vmax = fmaxf(vmax, fmaxf(__uint_as_float(u4[e] << 16), __uint_as_float(u4[e] & 0xFFFF0000u)));
                }
                *(uint4*)(o + c) = make_uint4(u4[0], u4[1], u4[2], u4[3]);
            }
        }
    }
    if constexpr (P::kFP8) {
        for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off));
        if ((threadIdx.x & 63) == 0) atomicMax(&a.amax_out[b], __float_as_uint(vmax));
    }
}

// Stem with stride 2 and max-pool 3/2 (two detectors, kernel 7) on the FP32
// matrix cores: per window the conv is an [L_conv x 16] x [16 x C] product,
// K = 2 channels x 8 taps (the eighth weight zero), as 16x16x4 MFMAs over
// 16-row blocks.  Conv rows go through LDS 256 at a time (ReLU applied) for
// the pool, whose window reaches one row into the previous pass; that row is
// carried over.  Every conv output is computed once.  One workgroup per
// window, samples staged in LDS as in stem2_kernel.
// Samples of a channel sit between zero pads: PADL before (>= the conv's 3)
// and PADR after, enough for the rows of a last, partial pass, so that the A
// operand reads need neither bounds checks nor selects.
struct StemMfmaGeom {
    static constexpr int RB = 4;              // 16-row blocks per wave per pass
    static constexpr int PR = 4 * RB * 16;    // conv rows per pass
    static constexpr int PADL = 4, PADR = 2 * PR + 8;
    static constexpr int pitch(int window) { return PADL + window + PADR; }
    static constexpr size_t lds_bytes(int window) { return (size_t)2 * pitch(window) * sizeof(float); }
};

template <typename P, int C>
__global__ void __launch_bounds__(256) stem_mfma_kernel(StemArgs a) {
    using Act = typename P::Act;
    using Geo = StemMfmaGeom;
    constexpr int KW = 7, PADS = 3, NCH = 2, S0 = 2;
    constexpr int NB = C / 16;          // 16-column blocks
    constexpr int RB = Geo::RB;
    constexpr int PR = Geo::PR;         // conv rows per pass
    constexpr int CP = C + 4;           // LDS row pitch (floats)
    static_assert(C % 16 == 0, "whole column blocks");
    __shared__ __attribute__((aligned(16))) float cb[(PR + 1) * CP];   // row 0: conv row before the pass
    extern __shared__ float xs[];       // [NCH][Geo::pitch(window)], samples at Geo::PADL
    const int b = blockIdx.x;
    const int64_t wi = a.first_window + b;
    const int W = a.window;
    const int XP = Geo::pitch(W);
    const WinAddr wa = window_addr(a, wi);
    for (int e = threadIdx.x; e < NCH * (Geo::PADL + Geo::PADR); e += 256) {   // zero pads
        const int c = e / (Geo::PADL + Geo::PADR), u = e % (Geo::PADL + Geo::PADR);
        xs[c * XP + (u < Geo::PADL ? u : W + u)] = 0.f;
    }
    stage_window(a, wa, xs, XP, Geo::PADL);   // a.n_ch == NCH
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    // B operand of k-step s for column block nb: k = 4s + g is channel k / 8, tap k % 8
    float bw[4][NB], bias[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        bias[nb] = a.b[nb * 16 + r16];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int k = 4 * st + g, ci = k >> 3, j = k & 7;
            bw[st][nb] = j < KW ? a.w[((nb * 16 + r16) * NCH + ci) * KW + j] : 0.f;
        }
    }
    for (int e = tid; e < CP; e += 256) cb[e] = 0.f;   // conv row -1 never wins (ReLU outputs are >= 0)
    __syncthreads();
    Act* out = (Act*)a.out + (size_t)b * a.L_out * C;
    constexpr int VE = 16 / (int)sizeof(Act);
    constexpr int VPR = C / VE;
    constexpr int NV = (PR / 2) * VPR;
    float vmax = 0.f;
    const int n_pass = (a.L_conv + PR - 1) / PR;
    for (int ps = 0; ps < n_pass; ++ps) {
        // all A operands of the pass first (clamped reads, zero padding by
        // select), then RB x NB independent accumulation chains
        // A operands of the pass: k = 4 st + g is channel st / 2, tap 4 (st & 1) + g
        // (tap 7 meets a zero weight); sample 2q - 3 + tap of the padded row
        float xa[RB][4];
        const float* xl = xs + Geo::PADL - PADS + 2 * (ps * PR + wv * RB * 16 + r16) + g;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int st = 0; st < 4; ++st) xa[rb][st] = xl[(st >> 1) * XP + 2 * 16 * rb + 4 * (st & 1)];
        f4v acc[RB][NB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = f4v{bias[nb], bias[nb], bias[nb], bias[nb]};
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[rb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[rb][st], bw[st][nb], acc[rb][nb], 0, 0, 0);
        // ReLU; rows past the conv output (a last, partial pass) are zero:
        // they never win the pool
        const bool full = (ps + 1) * PR <= a.L_conv;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = (wv * RB + rb) * 16 + g * 4 + r;
                    const float v = fmaxf(acc[rb][nb][r], 0.f);
                    cb[(1 + row) * CP + nb * 16 + r16] = (full || ps * PR + row < a.L_conv) ? v : 0.f;
                }
        __syncthreads();
        // pooled p = ps PR/2 + pl takes conv rows 2p - 1 .. 2p + 1, i.e. LDS rows 2pl .. 2pl + 2
        for (int v = tid; v < NV; v += 256) {
            const int pl = v / VPR, c0 = (v % VPR) * VE;
            const int p = ps * (PR / 2) + pl;
            if (p >= a.L_out) continue;
            float r[VE];
#pragma unroll
            for (int e = 0; e < VE; ++e)
                r[e] = fmaxf(fmaxf(cb[(2 * pl) * CP + c0 + e], cb[(2 * pl + 1) * CP + c0 + e]), cb[(2 * pl + 2) * CP + c0 + e]);
            Act* o = out + (size_t)p * C + c0;
            if constexpr (sizeof(Act) == 4) {
                *(float4*)o = make_float4(r[0], r[1], r[2], r[3]);
                vmax = fmaxf(vmax, fmaxf(fmaxf(r[0], r[1]), fmaxf(r[2], r[3])));
            } else {
                uint32_t u4[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    u4[e] = pack_bf16x2(r[2 * e], r[2 * e + 1]);
                    if constexpr (P::kFP8)
                        vmax = fmaxf(vmax, fmaxf(__uint_as_float(u4[e] << 16), __uint_as_float(u4[e] & 0xFFFF0000u)));
                }
                *(uint4*)o = make_uint4(u4[0], u4[1], u4[2], u4[3]);
            }
        }
        __syncthreads();
        for (int e = tid; e < CP; e += 256) cb[e] = cb[PR * CP + e];   // carry the pass's last conv row
        __syncthreads();
    }
    if constexpr (P::kFP8) {
        for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off));
        if ((threadIdx.x & 63) == 0) atomicMax(&a.amax_out[b], __float_as_uint(vmax));
    }
}

// Global average pool over time, then FC to one logit.  One workgroup of 256
// threads per window.  fc holds the C weights, then the bias.  A width C that
// divides 256 gives each channel 256 / C threads that stride over time; a
// width that is a multiple of 256 gives each thread C / 256 channels.  The
// FC products are reduced by wavefront shuffles, then across the four waves,
// always in the same order.
template <typename P>
__global__ void __launch_bounds__(256) gap_fc_kernel(const void* act, int L, int C, const float* fc,
                                                    float* logits) {
    using Act = typename P::Act;
    __shared__ float part[256];
    __shared__ float wpart[4];
    const int b = blockIdx.x, tid = threadIdx.x;
    const Act* x = (const Act*)act + (size_t)b * L * C;
    constexpr int U = 16;   // loads in flight per step
    float prod = 0.f;
    if (C <= 256) {
        const int per = 256 / C;
        const int c = tid % C, t0 = tid / C;
        float s = 0.f;
        for (int t = t0; t < L; t += per * U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // a clamped index past the end reads a valid element that then adds an exact zero
                const int tu = t + u * per;
                const float e = act_to_f32<P>(x[(size_t)(tu < L ? tu : L - 1) * C + c]);
                v[u] = tu < L ? e : 0.f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s += v[u];
        }
        part[tid] = s;
        __syncthreads();
        if (tid < C) {
            float tot = 0.f;
            for (int k = 0; k < per; ++k) tot += part[k * C + tid];
            prod = tot / (float)L * fc[tid];
        }
    } else {
        for (int c = tid; c < C; c += 256) {
            float s = 0.f;
            for (int t = 0; t < L; t += U) {
                float v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int tu = t + u;
                    const float e = act_to_f32<P>(x[(size_t)(tu < L ? tu : L - 1) * C + c]);
                    v[u] = tu < L ? e : 0.f;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) s += v[u];
            }
            prod += s / (float)L * fc[c];
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) prod += __shfl_xor(prod, off);
    if ((tid & 63) == 0) wpart[tid >> 6] = prod;
    __syncthreads();
    if (tid == 0) logits[b] = fc[C] + ((wpart[0] + wpart[1]) + (wpart[2] + wpart[3]));
}

// Per-channel sums of a [rows][C] FP32 tensor added into out[C] (FP64, one
// workgroup per channel, a fixed summation order).  Used to take the conv
// input means of a network during calibration.
__global__ void __launch_bounds__(256) channel_sum_kernel(const float* __restrict__ in, int64_t rows, int C,
                                                          double* __restrict__ out) {
    __shared__ double part[256];
    const int c = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int64_t r = tid; r < rows; r += 256) s += (double)in[r * C + c];
    part[tid] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) part[tid] += part[tid + o];
        __syncthreads();
    }
    if (tid == 0) out[c] += part[0];
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace afm
