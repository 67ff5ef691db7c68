// Kernels of the GroupNorm form of the scoring network (GroupNorm in place of
// BatchNorm, Sec. II).  GroupNorm normalises with statistics of the window
// being scored, so it cannot be folded into the weights: each conv of a block
// runs as the implicit-GEMM kernel with no bias and no ReLU and writes the
// statistics of its output as it stores it; gn_finalize_kernel turns them
// into per-channel scales and shifts; the block's second conv applies the
// first one's as it stages its input, and gn_apply_kernel ends the block
// (second norm, the projection's norm on the skip, residual add, ReLU).  The
// stem's norm runs inside the stem kernel.
#pragma once

#include "net_kernels.h"

namespace afm {

// The GroupNorm net's stem for any width C dividing 256: conv, GroupNorm,
// ReLU and (with a.pool) max-pool k3 s2 p1, one window per workgroup of 256
// threads, writing only the stem's output.  The conv (NCH x KW taps per
// output) is cheap, so it is computed twice instead of being stored.  Thread
// t takes channel t % C and the (t / C)-th of 256 / C consecutive row blocks.
// Pass 1 accumulates per-channel sums and sums of squares (FP32 over 16 rows,
// then FP64), reduced across the threads of a channel in block order, then
// per group in channel order; pass 2 recomputes each conv value where the
// output needs it, normalises it and applies ReLU, and the pool takes the
// maximum of rows 2p - 1 .. 2p + 1 (its last row is the next output's first,
// so it is computed once).  Samples are staged in LDS; weights in registers.
template <int NCH, int KW>
__global__ void __launch_bounds__(256) gn_stem_kernel(StemArgs a, const float* gamma, const float* beta, int G) {
    extern __shared__ float xs[];  // [n_ch][window]
    __shared__ double part[2][256];
    __shared__ float sc[256], sh[256];
    const int b = blockIdx.x, tid = threadIdx.x;
    const WinAddr wa = window_addr(a, a.first_window + b);
    stage_window(a, wa, xs);
    const int C = a.C, W = a.window, c = tid % C, rstep = 256 / C;
    float w[NCH][KW];
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci)
#pragma unroll
        for (int j = 0; j < KW; ++j) w[ci][j] = a.w[(c * NCH + ci) * KW + j];
    __syncthreads();
    constexpr int pad = (KW - 1) / 2;
    auto conv = [&](int t) {
        const int q0 = t * a.s0 - pad;
        float acc = 0.f;
#pragma unroll
        for (int ci = 0; ci < NCH; ++ci)
#pragma unroll
            for (int j = 0; j < KW; ++j) {
                const int q = q0 + j;
                const float x = (q >= 0 && q < W) ? xs[ci * W + q] : 0.f;
                acc = fmaf(w[ci][j], x, acc);
            }
        return acc;
    };
    const int rb = tid / C;
    const int nrow = (a.L_conv + rstep - 1) / rstep, r_lo = rb * nrow, r_hi = min(a.L_conv, r_lo + nrow);
    double s = 0.0, q = 0.0;
    for (int t0 = r_lo; t0 < r_hi; t0 += 16) {
        float fs = 0.f, fq = 0.f;
        const int t1 = min(t0 + 16, r_hi);
        for (int t = t0; t < t1; ++t) {
            const float v = conv(t);
            fs += v;
            fq = fmaf(v, v, fq);
        }
        s += (double)fs;
        q += (double)fq;
    }
    part[0][tid] = s;
    part[1][tid] = q;
    __syncthreads();
    if (tid < C) {
        // thread tid's channel sums: slots tid, tid + C, ... in order, then the group
        double cs = 0.0, cq = 0.0;
        for (int k = tid; k < 256; k += C) {
            cs += part[0][k];
            cq += part[1][k];
        }
        part[0][tid] = cs;   // slot tid was read above by this thread only
        part[1][tid] = cq;
    }
    __syncthreads();
    if (tid < C) {
        const int cpg = C / G, g = tid / cpg;
        double gs = 0.0, gq = 0.0;
        for (int cc = g * cpg; cc < (g + 1) * cpg; ++cc) {
            gs += part[0][cc];
            gq += part[1][cc];
        }
        const double n = (double)cpg * a.L_conv;
        const double mean = gs / n;
        const double var = fmax(gq / n - mean * mean, 0.0);
        const double scale = (double)gamma[tid] / sqrt(var + 1e-5);
        sc[tid] = (float)scale;
        sh[tid] = (float)((double)beta[tid] - mean * scale);
    }
    __syncthreads();
    const float S = sc[c], H = sh[c];
    float* out = (float*)a.out + (size_t)b * a.L_out * C;
    const int nout = (a.L_out + rstep - 1) / rstep, p_lo = rb * nout, p_hi = min(a.L_out, p_lo + nout);
    // ReLU of the normalised conv row r; rows outside the conv are 0 (every
    // pool candidate is >= 0)
    auto act = [&](int r) { return (r >= 0 && r < a.L_conv) ? fmaxf(fmaf(conv(r), S, H), 0.f) : 0.f; };
    if (a.pool) {
        float prev = p_lo < p_hi ? act(2 * p_lo - 1) : 0.f;
        for (int p = p_lo; p < p_hi; ++p) {
            const float r0 = act(2 * p), r1 = act(2 * p + 1);
            out[(size_t)p * C + c] = fmaxf(fmaxf(prev, r0), r1);
            prev = r1;
        }
    } else {
        for (int p = p_lo; p < p_hi; ++p) out[(size_t)p * C + c] = act(p);
    }
}

// The whole stem of the GroupNorm net in one pass, for 32-channel stems with a
// max-pool whose raw output has a multiple of 64 rows, at most 32 MAXR: raw
// conv -> GroupNorm -> ReLU -> max-pool k3 s2 p1, with the raw output held in
// registers.  1024 threads: thread t keeps channel t % 32 of the R = L_conv / 32
// consecutive rows of row block t / 32.  Statistics in FP64: a thread's R values,
// then across lanes l and l xor 32 (which share a channel), the 16 waves and
// the group's channels, in a fixed order.  Pooled row p of a block takes its
// rows 2p - 1 .. 2p + 1; the first of them for p = 0 is the previous block's last
// row, passed through LDS (row -1 is padding: every candidate is >= 0, so 0
// stands in for it).
template <int NCH, int KW, int MAXR>
__global__ void __launch_bounds__(1024) gn_stem_fused_kernel(StemArgs a, const float* gamma, const float* beta,
                                                             int G) {
    extern __shared__ float xs[];  // [n_ch][window]
    __shared__ double part[2][16][32];
    __shared__ double chs[2][32];
    __shared__ float sc[32], sh[32], edge[32][32];
    const int tid = threadIdx.x, c = tid & 31, rb = tid >> 5, lane = tid & 63, wv = tid >> 6;
    const int b = blockIdx.x;
    const WinAddr wa = window_addr(a, a.first_window + b);
    if (tid < 256) stage_window(a, wa, xs);
    const int W = a.window, R = a.L_conv / 32, r0 = rb * R;
    float w[NCH][KW];
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci)
#pragma unroll
        for (int j = 0; j < KW; ++j) w[ci][j] = a.w[(c * NCH + ci) * KW + j];
    __syncthreads();
    constexpr int pad = (KW - 1) / 2;
    float v[MAXR];
    double s = 0.0, q = 0.0;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
        v[i] = 0.f;
        if (i < R) {
            const int q0 = (r0 + i) * a.s0 - pad;
            float acc = 0.f;
#pragma unroll
            for (int ci = 0; ci < NCH; ++ci)
#pragma unroll
                for (int j = 0; j < KW; ++j) {
                    const int p = q0 + j;
                    const float x = (p >= 0 && p < W) ? xs[ci * W + p] : 0.f;
                    acc = fmaf(w[ci][j], x, acc);
                }
            v[i] = acc;
            s += (double)acc;
            q += (double)acc * (double)acc;
        }
    }
    s += __shfl_xor(s, 32);
    q += __shfl_xor(q, 32);
    if (lane < 32) {
        part[0][wv][c] = s;
        part[1][wv][c] = q;
    }
    __syncthreads();
    if (tid < 32) {
        double cs = 0.0, cq = 0.0;
        for (int k = 0; k < 16; ++k) {
            cs += part[0][k][tid];
            cq += part[1][k][tid];
        }
        chs[0][tid] = cs;
        chs[1][tid] = cq;
    }
    __syncthreads();
    if (tid < 32) {
        const int cpg = 32 / G, g = tid / cpg;
        double gs = 0.0, gq = 0.0;
        for (int cc = g * cpg; cc < (g + 1) * cpg; ++cc) {
            gs += chs[0][cc];
            gq += chs[1][cc];
        }
        const double n = (double)cpg * a.L_conv;
        const double mean = gs / n;
        const double var = fmax(gq / n - mean * mean, 0.0);
        const double scale = (double)gamma[tid] / sqrt(var + 1e-5);
        sc[tid] = (float)scale;
        sh[tid] = (float)((double)beta[tid] - mean * scale);
    }
    __syncthreads();
    const float S = sc[c], H = sh[c];
    float last = 0.f;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
        v[i] = fmaxf(fmaf(v[i], S, H), 0.f);
        if (i == R - 1) last = v[i];
    }
    edge[rb][c] = last;
    __syncthreads();
    const float prev = rb > 0 ? edge[rb - 1][c] : 0.f;
    float* out = (float*)a.out + (size_t)b * a.L_out * 32;
#pragma unroll
    for (int j = 0; j < MAXR / 2; ++j)
        if (2 * j < R) {
            const float left = j == 0 ? prev : v[2 * j - 1];
            out[(size_t)(rb * (R / 2) + j) * 32 + c] = fmaxf(fmaxf(left, v[2 * j]), v[2 * j + 1]);
        }
}

// GroupNorm scale and shift of one window per workgroup (256 threads) from
// the statistics the conv wrote: per channel, the sums and sums of squares of
// its nblk 16-row blocks are added in FP64, in block order (split over
// 256 / C strided parts when C < 256, the parts then added in order), then
// per group of C / G consecutive channels in channel order: mean, biased
// variance, scale_c = gamma_c / sqrt(var + eps), shift_c = beta_c -
// mean scale_c.  aff is [B][2][C] (scales, then shifts).
__global__ void __launch_bounds__(256) gn_finalize_kernel(const float* stats, int nblk, int L, int C, int G,
                                                          const float* gamma, const float* beta, float* aff) {
    __shared__ double part[2][1024];
    const int tid = threadIdx.x;
    const size_t b = blockIdx.x;
    const int per = C < 256 ? 256 / C : 1;
    const float* st = stats + b * nblk * 2 * C;
    for (int idx = tid; idx < per * C; idx += 256) {
        const int c = idx % C, pp = idx / C;
        // 8 blocks' values loaded before they are added (in block order; a
        // block past the end reads a valid one and adds an exact zero)
        constexpr int U = 8;
        double s = 0.0, q = 0.0;
        for (int k0 = pp; k0 < nblk; k0 += U * per) {
            float vs[U], vq[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + u * per < nblk ? k0 + u * per : pp;
                vs[u] = st[(size_t)k * 2 * C + c];
                vq[u] = st[(size_t)k * 2 * C + C + c];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = k0 + u * per < nblk;
                s += ok ? (double)vs[u] : 0.0;
                q += ok ? (double)vq[u] : 0.0;
            }
        }
        part[0][idx] = s;
        part[1][idx] = q;
    }
    __syncthreads();
    const int cpg = C / G;
    for (int c = tid; c < C; c += 256) {
        const int g = c / cpg;
        double gs = 0.0, gq = 0.0;
        for (int cc = g * cpg; cc < (g + 1) * cpg; ++cc)
            for (int pp = 0; pp < per; ++pp) {
                gs += part[0][pp * C + cc];
                gq += part[1][pp * C + cc];
            }
        const double n = (double)cpg * L;
        const double mean = gs / n;
        const double var = fmax(gq / n - mean * mean, 0.0);
        const double scale = (double)gamma[c] / sqrt(var + 1e-5);
        aff[b * 2 * C + c] = (float)scale;
        aff[b * 2 * C + C + c] = (float)((double)beta[c] - mean * scale);
    }
}

// out = relu(in scale + shift + r), r = res scale_r + shift_r (the residual's
// own GroupNorm, res_aff non-null) or res (res_aff null), or 0 (res null):
// the normalisation that ends a residual block.  Workgroup k takes slice
// k % n_slice of window k / n_slice: it stages the window's scales and shifts
// in LDS and takes U float4s per thread of the slice.  Each element is read and written by one thread,
// so out may alias in or res.
struct GnApplyArgs {
    const float* in;        // [B][L][C]
    const float* res;       // [B][L][C] or null
    float* out;             // [B][L][C]
    const float* aff;       // [B][2][C]
    const float* res_aff;   // [B][2][C] or null
    int LC4, C;             // float4s per window, channels (a multiple of 4, at most 1024)
    int relu;
    int n_slice;            // workgroups per window: ceil(LC4 / (256 U))
};
template <int U>
__global__ void __launch_bounds__(256) gn_apply_kernel(GnApplyArgs a) {
    __shared__ float4 saff[2][256], raff[2][256];
    const int tid = threadIdx.x, C4 = a.C >> 2;
    const size_t b = blockIdx.x / a.n_slice;
    const int slice = (int)(blockIdx.x % a.n_slice);
    for (int c = tid; c < C4; c += 256) {
        saff[0][c] = ((const float4*)(a.aff + b * 2 * a.C))[c];
        saff[1][c] = ((const float4*)(a.aff + b * 2 * a.C + a.C))[c];
        if (a.res_aff) {
            raff[0][c] = ((const float4*)(a.res_aff + b * 2 * a.C))[c];
            raff[1][c] = ((const float4*)(a.res_aff + b * 2 * a.C + a.C))[c];
        }
    }
    __syncthreads();
    const float4* in = (const float4*)a.in + b * a.LC4;
    const float4* res = a.res ? (const float4*)a.res + b * a.LC4 : nullptr;
    float4* out = (float4*)a.out + b * a.LC4;
    const int i0 = slice * 256 * U + tid;
    float4 v[U], r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = min(i0 + 256 * u, a.LC4 - 1);
        v[u] = in[i];
        r[u] = res ? res[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    auto fma4 = [](float4 x, float4 m, float4 c) {
        return make_float4(fmaf(x.x, m.x, c.x), fmaf(x.y, m.y, c.y), fmaf(x.z, m.z, c.z), fmaf(x.w, m.w, c.w));
    };
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = i0 + 256 * u;
        if (i >= a.LC4) break;
        const int c4 = i % C4;
        float4 y = fma4(v[u], saff[0][c4], saff[1][c4]);
        if (res) {
            const float4 rr = a.res_aff ? fma4(r[u], raff[0][c4], raff[1][c4]) : r[u];
            y = make_float4(y.x + rr.x, y.y + rr.y, y.z + rr.z, y.w + rr.w);
        }
        if (a.relu) y = make_float4(fmaxf(y.x, 0.f), fmaxf(y.y, 0.f), fmaxf(y.z, 0.f), fmaxf(y.w, 0.f));
        out[i] = y;
    }
}

}  // namespace afm
