// Whole-network kernel for the 16-channel, two-block ResNet (stem k7 s1, two
// BasicBlocks of 16 channels, GAP, FC) in BF16: one wavefront per window,
// persistent over windows.
//
// Workgroups take windows from a queue: the first window of workgroup b is
// window b, the next ones come from an atomic counter (cleared before the
// launch), so the launch may hold more workgroups than fit the device at once
// without leaving late ones a full share of the work.
//
// A wavefront walks its window in steps of T time rows.  In step k the stem
// produces rows [kT, kT + T) and conv layer l (l = 1..4) the rows
// [kT - 3l, kT + T - 3l).  A k7 conv reads 3 rows beyond its output on each
// side; the layer before produced them in this step or in the previous one,
// whose last 6 rows every buffer carries to its front, so no row is computed
// twice.  Rows outside the window are forced to zero (the per-layer zero
// padding of the unfused network); only the steps that reach outside the
// window (the first and the last) test rows at all.  Activations stay in the
// wavefront's LDS (BF16), weights in registers.  With one wavefront per
// workgroup, ordering its own LDS accesses between layers needs no barrier,
// only a wait for its LDS operations (wave_lds_sync); the next step's input
// loads stay in flight meanwhile.
//
// Every layer runs on the matrix cores, transposed (D[channel][time] =
// W[channel][k] X[k][time]) in 16-row tiles, so that a lane ends with four
// consecutive channels of one time row:
//  - stem: FP32 16x16x4 MFMAs over k = input channel x 8 + tap (the eighth
//    tap has weight 0), FP32 weights and input;
//  - convs: BF16 16x16x32 MFMAs over k = tap x 16 + channel.  The eighth tap
//    pads K from 112 to 128; in the second conv of a block it carries the
//    residual (identity weights times the block input's row), which is then
//    summed in FP32 with the products.  Each k-step's operands are read from
//    LDS two k-steps ahead of their MFMAs (the stem's all at once);
//  - the bias is the accumulator's initial value.
// Outputs are rounded to BF16 (hardware round-to-nearest-even) and then
// passed through ReLU as packed 16-bit integers (a BF16 value is negative iff
// its bit pattern is, and rounding commutes with max(., 0)); the second
// block's output goes to the global average, then FC.
#pragma once
#include <type_traits>

#include "net_kernels.h"

namespace afm {

struct FusedTinyArgs {
    StemArgs st;               // window addressing and window length
    const float* wstem;        // [16][16]: output channel, k = input channel * 8 + tap (tap 7: 0)
    const uint16_t* wconv;     // [4][16][128] BF16, k = tap * 16 + channel; tap 7 as described above
    const float* bias;         // [5][16]: stem, then the four convs
    const float* fc;           // [16] weights, then the bias
    float* logits;
    int64_t n_windows;
    unsigned int* next;        // window queue counter (zero at launch)
};

// Orders this wavefront's LDS accesses across the point: stores before it
// are seen by loads after it in every lane of the wavefront.  A wavefront's
// LDS operations execute in issue order, so this needs no wait in the
// instruction stream: wavefront-scope release and acquire fences around a
// wave barrier keep the compiler from moving accesses across it.  Global
// loads in flight are not waited for.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// BF16 pair: round to nearest even, then ReLU on the bit patterns (one packed
// signed 16-bit max).
typedef short short2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu_bf16x2(float lo, float hi) {
    const short2v v = __builtin_bit_cast(short2v, pack_bf16x2(lo, hi));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, short2v{0, 0}));
}
// A tile's four outputs (channels 4g .. 4g + 3 of one time row t) as stored;
// with EDGE, zero when t lies outside [0, L).
template <bool EDGE>
__device__ __forceinline__ uint2 finish_tile(const f4v& acc, int t, int L) {
    uint2 p = make_uint2(relu_bf16x2(acc[0], acc[1]), relu_bf16x2(acc[2], acc[3]));
    if (EDGE && (t < 0 || t >= L)) p = make_uint2(0u, 0u);
    return p;
}

namespace fused_tiny {
constexpr int C = 16;
constexpr int TAIL = 6;         // rows carried from step to step
template <int T, int PITCH>
struct Geo {
    static constexpr int ROWS = T + TAIL;      // rows per activation buffer
    static constexpr int BUF = ROWS * PITCH;   // elements per buffer
    static constexpr int XN = T + TAIL;        // input samples per channel
};
}  // namespace fused_tiny

// Element offset of channel half `hf` (8 channels, 16 bytes) of activation
// row t.  SWZ: 64-byte rows whose 16-byte units are XOR-swizzled by
// (t / 2) & 3 (the layout the MFMA operand reads meet without LDS bank
// conflicts); otherwise plain rows of PITCH elements.
template <int PITCH, bool SWZ>
__device__ __forceinline__ int act_off(int t, int hf) {
    return t * PITCH + 8 * (SWZ ? (hf ^ ((t >> 1) & 3)) : hf);
}

// T: time rows per step; PITCH: BF16 elements per stored activation row (16
// channels and padding); SWZ: the swizzled 64-byte rows (PITCH 32).
// Sample indices are 32-bit: the caller guarantees n_ch * ld_y < 2^31.
template <int T, int PITCH, bool SWZ>
__global__ void __launch_bounds__(64, 3) fused_tiny_bf16_kernel(FusedTinyArgs a) {
    using namespace fused_tiny;
    using G = Geo<T, PITCH>;
    static_assert(!SWZ || (PITCH == 32 && T % 8 == 0), "the swizzle needs 4 units per row and whole periods per step");
    constexpr int UPR = PITCH / 8;              // 16-byte units per stored row
    static_assert(T % 16 == 0 && T <= 64, "steps of whole 16-row tiles");
    constexpr int NT = T / 16;                  // 16-row tiles per step
    __shared__ __attribute__((aligned(16))) uint16_t act[4 * G::BUF];   // stem, conv 1, conv 2, conv 3 outputs
    __shared__ float xs[2 * G::XN];
    __shared__ __attribute__((aligned(16))) float sbias[5 * C];   // read per layer and step: fewer live registers
    const int lane = threadIdx.x, g = lane >> 4, r16 = lane & 15;
    const int L = a.st.window;

    // weights for the kernel's lifetime
    float ws[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) ws[s] = a.wstem[r16 * 16 + 4 * s + g];
    bf16x8 wa[4][4];
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int s = 0; s < 4; ++s)
            wa[l][s] = *(const bf16x8*)(a.wconv + ((size_t)l * C + r16) * 128 + 32 * s + 8 * g);
    for (int e = lane; e < 5 * C; e += 64) sbias[e] = a.bias[e];
    auto bias = [&](int l) { return *(const f4v*)(sbias + l * C + 4 * g); };
    auto buf = [&](int b) { return act + b * G::BUF; };
    // the carried rows: 4 buffers x TAIL rows x UPR 16-byte units, at most two
    // per lane; their element offsets (front of the buffer) are fixed
    constexpr int NCARRY = 4 * TAIL * UPR;
    static_assert(NCARRY <= 128, "two carried units per lane at most");
    int coff[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int e = lane + 64 * i, b = e / (TAIL * UPR), u = e % (TAIL * UPR);
        coff[i] = b * G::BUF + (u / UPR) * PITCH + (u % UPR) * 8;
    }
    const int nsteps = (L + 12 + T - 1) / T;

    int64_t win = blockIdx.x;
    while (win < a.n_windows) {
        // the window after this one, asked for now and used at the end
        unsigned int ticket = 0;
        if (lane == 0) ticket = atomicAdd(a.next, 1u);
        // sample t of channel c is y[e0[c] + t], less `wrap` from t = lim[c] on
        const WinAddr wad = window_addr(a.st, win);
        int e0[2], lim[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            e0[c] = (int)(c * a.st.ld_y + wad.base + wad.start[c]);
            lim[c] = wad.wrap > 0 ? (int)(wad.wrap - wad.start[c]) : 0x7FFFFFFF;
        }
        const int wrap = (int)wad.wrap;
        auto sample = [&](int c, int t) -> float {
            const int e = e0[c] + t - (t >= lim[c] ? wrap : 0);
            return (t >= 0 && t < L) ? a.st.y[e] : 0.f;
        };
        // window start: the carried rows lie before the window (zero); the
        // input's carried samples are those of times -3 .. 2
#pragma unroll
        for (int i = 0; i < 2; ++i)
            if (lane + 64 * i < NCARRY) *(uint4*)(act + coff[i]) = make_uint4(0u, 0u, 0u, 0u);
        if (lane < 2 * TAIL) xs[(lane / TAIL) * G::XN + lane % TAIL] = sample(lane / TAIL, lane % TAIL - 3);
        // samples of times s0 + 3 .. s0 + T + 2 of step 0
        float nx[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) nx[c] = lane < T ? sample(c, 3 + lane) : 0.f;
        f4v gs = {0.f, 0.f, 0.f, 0.f};

        // one step; EDGE (the first and last steps) zeroes rows outside the window
        auto step = [&](const int k, auto edge_tag) {
            constexpr bool EDGE = decltype(edge_tag)::value;
            const int s0 = k * T;
            if (lane < T) {
                xs[TAIL + lane] = nx[0];
                xs[G::XN + TAIL + lane] = nx[1];
            }
            // the next step's samples are loaded now and stored a step later
            if (k + 1 < nsteps) {
#pragma unroll
                for (int c = 0; c < 2; ++c) nx[c] = lane < T ? sample(c, s0 + T + 3 + lane) : 0.f;
            }
            wave_lds_sync();

            // ---- stem: rows s0 .. s0 + T - 1 into buffer 0 (rows TAIL ..)
            {
                const float* xb[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int j = 4 * (s & 1) + g;   // k = 4s + g: input channel s / 2, tap j
                    xb[s] = xs + (s >> 1) * G::XN + r16 + (j == 7 ? 6 : j);   // tap 7: any sample, weight 0
                }
                f4v acc[NT];
#pragma unroll
                for (int m = 0; m < NT; ++m) acc[m] = bias(0);
                // every operand read before the first product (the scheduler
                // would otherwise wait for each k-step's reads in turn)
                float xv[4][NT];
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int m = 0; m < NT; ++m) xv[s][m] = xb[s][16 * m];
                __builtin_amdgcn_sched_barrier(0);
                // raised issue priority while the products run: a wavefront
                // with MFMAs ready goes before the others' LDS and VALU work
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int m = 0; m < NT; ++m) acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(ws[s], xv[s][m], acc[m], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(0);
                // row TAIL + 16m + r16 keeps the swizzle phase of TAIL + r16
                const int so = act_off<PITCH, SWZ>(TAIL + r16, g >> 1) + 4 * (g & 1);
#pragma unroll
                for (int m = 0; m < NT; ++m)
                    *(uint2*)(buf(0) + so + 16 * m * PITCH) = finish_tile<EDGE>(acc[m], s0 + 16 * m + r16, L);
            }
            wave_lds_sync();

            // ---- conv layer l: buffer l -> buffer l + 1 (or the average)
            // layer l (a compile-time constant): the second conv of a block
            // (l odd) reads the block input as its eighth tap; the last one
            // feeds the global average instead of a buffer
            auto conv = [&](auto lc, const uint16_t* in, const uint16_t* res, uint16_t* out) {
                constexpr int l = decltype(lc)::value;
                constexpr bool RES = (l & 1) != 0, GAP = l == 3;
                const uint16_t* bsrc[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int j = 2 * s + (g >> 1), hf = g & 1;
                    if (RES)
                        bsrc[s] = j < 7 ? in + act_off<PITCH, SWZ>(r16 + j, hf) : res + act_off<PITCH, SWZ>(r16, hf);
                    else
                        bsrc[s] = in + act_off<PITCH, SWZ>(r16 + (j < 7 ? j : 6), hf);
                }
                f4v acc[NT];
#pragma unroll
                for (int m = 0; m < NT; ++m) acc[m] = bias(l + 1);
                // operands read LA k-steps ahead of their products, in a ring
                // of LA + 1; the scheduling barriers keep that order (left
                // alone, the scheduler issues each k-step's reads only after
                // the previous k-step's products and then waits for them)
                constexpr int LA = 2;   // three ahead measured no faster, one 3 % slower
                bf16x8 xv[LA + 1][NT];
#pragma unroll
                for (int s = 0; s < LA; ++s)
#pragma unroll
                    for (int m = 0; m < NT; ++m) xv[s][m] = *(const bf16x8*)(bsrc[s] + 16 * m * PITCH);
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int s = 0; s < 4; ++s) {
#pragma unroll
                    for (int m = 0; m < NT; ++m)
                        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[l][s], xv[s % (LA + 1)][m], acc[m], 0, 0, 0);
                    if (s + LA < 4) {
#pragma unroll
                        for (int m = 0; m < NT; ++m)
                            xv[(s + LA) % (LA + 1)][m] = *(const bf16x8*)(bsrc[s + LA] + 16 * m * PITCH);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                __builtin_amdgcn_s_setprio(0);
                const int tl = s0 - 3 * (l + 1);   // time of output row 0
                const int so = act_off<PITCH, SWZ>(TAIL + r16, g >> 1) + 4 * (g & 1);
#pragma unroll
                for (int m = 0; m < NT; ++m) {
                    const uint2 packed = finish_tile<EDGE>(acc[m], tl + 16 * m + r16, L);
                    if constexpr (!GAP) {
                        *(uint2*)(out + so + 16 * m * PITCH) = packed;
                    } else {
                        gs[0] += __uint_as_float(packed.x << 16);
                        gs[1] += __uint_as_float(packed.x & 0xFFFF0000u);
                        gs[2] += __uint_as_float(packed.y << 16);
                        gs[3] += __uint_as_float(packed.y & 0xFFFF0000u);
                    }
                }
            };
            conv(std::integral_constant<int, 0>{}, buf(0), nullptr, buf(1));   // block 0 conv1
            wave_lds_sync();
            conv(std::integral_constant<int, 1>{}, buf(1), buf(0), buf(2));    // block 0 conv2 + block input
            wave_lds_sync();
            conv(std::integral_constant<int, 2>{}, buf(2), nullptr, buf(3));   // block 1 conv1
            wave_lds_sync();
            conv(std::integral_constant<int, 3>{}, buf(3), buf(2), nullptr);   // block 1 conv2 + block input -> average
            wave_lds_sync();

            // carry the last TAIL rows of every buffer, and of the input, to the front
#pragma unroll
            for (int i = 0; i < 2; ++i)   // whole rows: T keeps the swizzle phase
                if (lane + 64 * i < NCARRY) *(uint4*)(act + coff[i]) = *(const uint4*)(act + coff[i] + T * PITCH);
            if (lane < 2 * TAIL) xs[(lane / TAIL) * G::XN + lane % TAIL] = xs[(lane / TAIL) * G::XN + T + lane % TAIL];
            wave_lds_sync();
        };
        for (int k = 0; k < nsteps; ++k) {
            // a step reaches outside the window when layer 4 starts before time
            // 0 or the stem ends past the last sample
            if (k * T < 12 || (k + 1) * T > L)
                step(k, std::true_type{});
            else
                step(k, std::false_type{});
        }
        // global average (sum over the lane's rows, then over the 16 lanes of
        // each channel group) and FC, in a fixed order
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) gs[r] += __shfl_xor(gs[r], off);
        float z = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) z += gs[r] / (float)L * a.fc[4 * g + r];
        z += __shfl_xor(z, 16);
        z += __shfl_xor(z, 32);
        if (lane == 0) a.logits[win] = a.fc[C] + z;
        wave_lds_sync();
        win = (int64_t)gridDim.x + (int64_t)__shfl(ticket, 0);
    }
}

}  // namespace afm
