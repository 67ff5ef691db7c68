// Whole-network kernel for the 16-channel, two-block ResNet (stem k7 s1,
// two BasicBlocks of 16 channels, GAP, FC) in BF16, persistent over windows.
//
// Each workgroup walks windows g = blockIdx.x, blockIdx.x + gridDim.x, ...
// (every wave leaves the loop when g passes n_windows).  A window is processed
// in time tiles of T = 232 outputs.  The tile's 256 rows cover times
// t0 - 12 ... t0 + T + 11: the four k7 convs each shrink the valid range by 3
// rows per side, so the last layer is valid on [t0, t0 + T).  Rows outside the
// window are forced to zero after every layer, which is the per-layer zero
// padding of the unfused network.  All activations stay in LDS (BF16); the
// four conv weight matrices stay in registers for the workgroup's lifetime.
//
// Each conv is computed transposed on 16x16x32 BF16 MFMA tiles:
// D[channel][time] = W[channel][k] * X[k][time], k = tap * 16 + channel_in
// (tap 7 is a zero pad that brings K = 112 to 128), so that a lane ends up with
// four consecutive output channels of one time row and stores them as 8 bytes.
#pragma once
#include "net_kernels.h"

namespace afm {

struct FusedTinyArgs {
    StemArgs st;               // addressing + stem weights (FP32), window length
    const uint16_t* wconv;     // [4][16][128] BF16, layer-major, k = tap*16 + c
    const float* bconv;        // [4][16]
    const float* fc_w;         // [16]
    float fc_b;
    float* logits;
    int64_t n_windows;
};

namespace fused_tiny {
constexpr int C = 16;
constexpr int R = 256;          // rows per tile (one per thread for the stem)
constexpr int HALO = 12;        // 4 convs x 3
constexpr int T = R - 2 * HALO; // valid outputs per tile
constexpr int XR = R + 6;       // input samples per tile and channel
constexpr int PITCH = 24;       // BF16 elements per activation row (48 B: conflict-free 16 B reads)
constexpr int GUARD = 3;        // rows before row 0
constexpr int ROWS = R + 8;     // GUARD + R + 5 (tap 7 reads row q + 7)
constexpr int BUF = ROWS * PITCH;
}  // namespace fused_tiny

__global__ void __launch_bounds__(256) fused_tiny_bf16_kernel(FusedTinyArgs a) {
    using namespace fused_tiny;
    __shared__ __attribute__((aligned(16))) uint16_t act[3 * BUF];
    __shared__ float xs[2 * XR];
    __shared__ float gpart[4 * C];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int L = a.st.window;

    // zero the guard rows once; tiles only ever write rows GUARD .. GUARD + R - 1
    for (int e = tid; e < 3 * 8 * PITCH; e += 256) {
        const int b = e / (8 * PITCH), rr = (e / PITCH) % 8, c = e % PITCH;
        const int row = rr < GUARD ? rr : R + rr;   // rows 0..2 and R+3..R+7
        act[b * BUF + row * PITCH + c] = 0;
    }
    // conv weights (A operand) for all four layers and bias
    bf16x8 wa[4][4];
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int s = 0; s < 4; ++s)
            wa[l][s] = *(const bf16x8*)(a.wconv + ((size_t)l * C + r16) * 128 + 32 * s + 8 * g);
    float bias[4][4];
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[l][r] = a.bconv[l * C + 4 * g + r];
    __syncthreads();

    uint16_t* bufA = act;
    uint16_t* bufB = act + BUF;
    uint16_t* bufC = act + 2 * BUF;

    for (int64_t win = blockIdx.x; win < a.n_windows; win += gridDim.x) {
        const WinAddr wad = window_addr(a.st, win);
        float gsum[4] = {0.f, 0.f, 0.f, 0.f};
        for (int t0 = 0; t0 < L; t0 += T) {
            // stage the input samples t0 - 15 ... t0 + T + 14 of both detectors
            for (int e = tid; e < 2 * XR; e += 256) {
                const int ci = e / XR, u = e % XR;
                const int t = t0 - HALO - 3 + u;
                xs[e] = (t >= 0 && t < L) ? a.st.y[ci * a.st.ld_y + window_sample(wad, ci, t)] : 0.f;
            }
            __syncthreads();
            // stem: row q = tid, time t0 - 12 + q, all 16 channels (FP32, stored BF16)
            {
                const int q = tid, t = t0 - HALO + q;
                float xin[2][7];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                    for (int j = 0; j < 7; ++j) xin[ci][j] = xs[ci * XR + q + j];
                const bool inside = t >= 0 && t < L;
                uint32_t packed[C / 2];
#pragma unroll
                for (int c = 0; c < C; c += 2) {
                    float v[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        float sacc = a.st.b[c + h];
#pragma unroll
                        for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                            for (int j = 0; j < 7; ++j) sacc = fmaf(a.st.w[((c + h) * 2 + ci) * 7 + j], xin[ci][j], sacc);
                        v[h] = inside ? fmaxf(sacc, 0.f) : 0.f;
                    }
                    packed[c / 2] = pack_bf16x2(v[0], v[1]);
                }
                uint4* dst = (uint4*)(bufA + (q + GUARD) * PITCH);
                dst[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
                dst[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
            }
            __syncthreads();

            // one conv layer: in -> out (or GAP when out == null); residual optional
            auto layer = [&](int l, const uint16_t* in, uint16_t* out, const uint16_t* res) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int q0 = (wave * 4 + m) * 16;     // first row of this 16-row tile
                    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int k0 = 32 * s + 8 * g;
                        const int j = k0 >> 4, c0 = k0 & 15;
                        const bf16x8 xb = *(const bf16x8*)(in + (q0 + r16 + j) * PITCH + c0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[l][s], xb, acc, 0, 0, 0);
                    }
                    const int q = q0 + r16, t = t0 - HALO + q;
                    const bool inside = t >= 0 && t < L;
                    float v[4];
                    uint2 rres = make_uint2(0u, 0u);
                    if (res) rres = *(const uint2*)(res + (q + GUARD) * PITCH + 4 * g);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float x = acc[r] + bias[l][r];
                        if (res) {
                            const uint32_t w2 = r < 2 ? rres.x : rres.y;
                            x += __uint_as_float((r & 1) ? (w2 & 0xFFFF0000u) : (w2 << 16));
                        }
                        x = inside ? fmaxf(x, 0.f) : 0.f;
                        v[r] = bf16_bits_to_f32(f32_to_bf16_bits(x));
                    }
                    if (out) {
                        const uint32_t lo = (__float_as_uint(v[0]) >> 16) | (__float_as_uint(v[1]) & 0xFFFF0000u);
                        const uint32_t hi = (__float_as_uint(v[2]) >> 16) | (__float_as_uint(v[3]) & 0xFFFF0000u);
                        *(uint2*)(out + (q + GUARD) * PITCH + 4 * g) = make_uint2(lo, hi);
                    } else if (t >= t0 && t < t0 + T && t < L) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) gsum[r] += v[r];
                    }
                }
            };
            layer(0, bufA, bufB, nullptr);   // block 0 conv1: h0 -> r1
            __syncthreads();
            layer(1, bufB, bufC, bufA);      // block 0 conv2 + h0: -> h2
            __syncthreads();
            layer(2, bufC, bufB, nullptr);   // block 1 conv1: h2 -> r3
            __syncthreads();
            layer(3, bufB, nullptr, bufC);   // block 1 conv2 + h2: -> GAP
            __syncthreads();
        }
        // GAP: sum the 16 rows held by the lanes of each group, then the waves
#pragma unroll
        for (int r = 0; r < 4; ++r)
            for (int off = 8; off > 0; off >>= 1) gsum[r] += __shfl_xor(gsum[r], off);
        if (r16 == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) gpart[wave * C + 4 * g + r] = gsum[r];
        }
        __syncthreads();
        if (tid == 0) {
            float z = a.fc_b;
            for (int c = 0; c < C; ++c) {
                const float tot = ((gpart[c] + gpart[C + c]) + gpart[2 * C + c]) + gpart[3 * C + c];
                z += tot / (float)L * a.fc_w[c];
            }
            a.logits[win] = z;
        }
        __syncthreads();
    }
}

}  // namespace afm
