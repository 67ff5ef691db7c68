// Kernels of the GroupNorm form of the scoring network (GroupNorm in place of
// BatchNorm, Sec. II).  GroupNorm normalises with statistics of the window
// being scored, so it cannot be folded into the convolutions: each conv runs
// as the implicit-GEMM kernel with no bias and no ReLU, and gn_kernel then
// normalises its output.
#pragma once

#include "net_kernels.h"

namespace afm {

// Raw stem conv: out[b][t][c] = sum over input channels ci and taps j of
// w[c][ci][j] x_ci[t s0 + j - (KW-1)/2] (zero outside the window), FP32
// vector arithmetic, no bias, no ReLU, no pool; out is [B][L_conv][C].  C
// divides 256, so each thread keeps one channel (its weights in registers)
// and steps through the rows 256 / C at a time.
template <int NCH, int KW>
__global__ void __launch_bounds__(256) gn_stem_kernel(StemArgs a) {
    extern __shared__ float xs[];  // [n_ch][window]
    const int b = blockIdx.x;
    const WinAddr wa = window_addr(a, a.first_window + b);
    stage_window(a, wa, xs);
    const int C = a.C, W = a.window, c = threadIdx.x % C, rstep = 256 / C;
    float w[NCH][KW];
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci)
#pragma unroll
        for (int j = 0; j < KW; ++j) w[ci][j] = a.w[(c * NCH + ci) * KW + j];
    __syncthreads();
    constexpr int pad = (KW - 1) / 2;
    float* out = (float*)a.out + (size_t)b * a.L_conv * C;
    for (int t = threadIdx.x / C; t < a.L_conv; t += rstep) {
        const int q0 = t * a.s0 - pad;
        float s = 0.f;
#pragma unroll
        for (int ci = 0; ci < NCH; ++ci)
#pragma unroll
            for (int j = 0; j < KW; ++j) {
                const int q = q0 + j;
                const float x = (q >= 0 && q < W) ? xs[ci * W + q] : 0.f;
                s = fmaf(w[ci][j], x, s);
            }
        out[(size_t)t * C + c] = s;
    }
}

// The whole stem of the GroupNorm net in one pass, for 32-channel stems with a
// max-pool whose raw output has a multiple of 64 rows, at most 32 MAXR: raw
// conv -> GroupNorm -> ReLU -> max-pool k3 s2 p1, with the raw output held in
// registers.  1024 threads: thread t keeps channel t % 32 of the R = L_conv / 32
// consecutive rows of row block t / 32.  Statistics as in gn_reg_kernel (lanes
// l and l xor 32 share a channel).  Pooled row p of a block takes its rows
// 2p - 1 .. 2p + 1; the first of them for p = 0 is the previous block's last
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

struct GnArgs {
    const float* in;      // [B][L][C]
    const float* res;     // [B][L][C] added after the affine map, or null
    float* out;           // [B][L_out][C]; may alias in or res when pool == 0
    const float* gamma;   // [C]
    const float* beta;    // [C]
    int L, C, G;          // C a power of two in [16, 1024], G divides C
    int relu;             // ReLU after the (residual) add
    int pool;             // max-pool k3 s2 p1 after the ReLU (relu must be set)
};

// GroupNorm of one window per workgroup (256 threads).  Pass 1: per-channel
// sums and sums of squares in FP64 (1024 is a multiple of C, so a thread's
// four channels stay fixed as it strides through the window's float4s),
// reduced per group in a fixed order: mean and biased variance, for channels
// tid, tid + 256, ... .  Pass 2:
// v * scale_c + shift_c with scale_c = gamma_c / sqrt(var_g + eps),
// shift_c = beta_c - mean_g scale_c, then residual add, ReLU, pool.  Each
// element of `out` is written by the thread that read it in pass 2, and pass 1
// ends at a barrier, so out may alias in or res.
__global__ void __launch_bounds__(256) gn_kernel(GnArgs a) {
    constexpr int U = 8;   // float4 loads in flight per thread
    __shared__ double part[2][1024];
    __shared__ float sc[1024], sh[1024];
    const int tid = threadIdx.x, C = a.C, L = a.L;
    const size_t b = blockIdx.x;
    const float4* in = (const float4*)(a.in + b * L * C);
    const int n4 = L * C / 4;
    double s[4] = {0.0, 0.0, 0.0, 0.0}, q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i0 = tid; i0 < n4; i0 += 256 * U) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = in[min(i0 + 256 * u, n4 - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + 256 * u >= n4) break;
            const float e[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[k] += (double)e[k];
                q[k] += (double)e[k] * (double)e[k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        part[0][4 * tid + k] = s[k];
        part[1][4 * tid + k] = q[k];
    }
    __syncthreads();
    // slot p of part holds channel p % C; channel c of group g = c / (C / G)
    for (int ch = tid; ch < C; ch += 256) {
        const int cpg = C / a.G, g = ch / cpg;
        double gs = 0.0, gq = 0.0;
        for (int c = g * cpg; c < (g + 1) * cpg; ++c)
            for (int p = c; p < 1024; p += C) {
                gs += part[0][p];
                gq += part[1][p];
            }
        const double n = (double)cpg * L;
        const double mean = gs / n;
        const double var = fmax(gq / n - mean * mean, 0.0);
        const double scale = (double)a.gamma[ch] / sqrt(var + 1e-5);
        sc[ch] = (float)scale;
        sh[ch] = (float)((double)a.beta[ch] - mean * scale);
    }
    __syncthreads();
    const int c0 = (4 * tid) % C;
    const float4 S = make_float4(sc[c0], sc[c0 + 1], sc[c0 + 2], sc[c0 + 3]);
    const float4 H = make_float4(sh[c0], sh[c0 + 1], sh[c0 + 2], sh[c0 + 3]);
    auto norm = [&](float4 v) {
        return make_float4(fmaf(v.x, S.x, H.x), fmaf(v.y, S.y, H.y), fmaf(v.z, S.z, H.z), fmaf(v.w, S.w, H.w));
    };
    auto relu4 = [](float4 v) {
        return make_float4(fmaxf(v.x, 0.f), fmaxf(v.y, 0.f), fmaxf(v.z, 0.f), fmaxf(v.w, 0.f));
    };
    if (!a.pool) {
        const float4* res = a.res ? (const float4*)(a.res + b * L * C) : nullptr;
        float4* out = (float4*)(a.out + b * L * C);
        for (int i0 = tid; i0 < n4; i0 += 256 * U) {
            float4 v[U], r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = min(i0 + 256 * u, n4 - 1);
                v[u] = in[i];
                r[u] = res ? res[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i0 + 256 * u >= n4) break;
                float4 y = norm(v[u]);
                if (res) y = make_float4(y.x + r[u].x, y.y + r[u].y, y.z + r[u].z, y.w + r[u].w);
                out[i0 + 256 * u] = a.relu ? relu4(y) : y;
            }
        }
    } else {
        // pooled row p takes rows 2p-1, 2p, 2p+1 of the normalised, ReLU'd
        // input; every candidate is >= 0, so 0 starts the max
        const int L_out = (L - 1) / 2 + 1, C4 = C / 4;
        const int n4o = L_out * C4;
        float4* out = (float4*)(a.out + b * L_out * C);
        for (int i = tid; i < n4o; i += 256) {
            const int p = i / C4, cq = i - p * C4;
            float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int r = 2 * p - 1; r <= 2 * p + 1; ++r) {
                if (r < 0 || r >= L) continue;
                const float4 y = relu4(norm(in[r * C4 + cq]));
                m = make_float4(fmaxf(m.x, y.x), fmaxf(m.y, y.y), fmaxf(m.z, y.z), fmaxf(m.w, y.w));
            }
            out[i] = m;
        }
    }
}

// GroupNorm of one window per workgroup with the window held in registers
// (no pool): NT threads, up to R float4s each, so a window of up to 4 NT R
// elements is read from HBM once instead of twice, for C <= 256.  Each
// thread's channels are fixed (C divides 4 NT); its sums and sums of squares per channel (FP32,
// R terms each) are reduced in FP64 across the lanes that share channels (lane xor C/4 .. 32), then
// across the NT / 64 waves and per group in a fixed order.  Then as gn_kernel:
// scale, shift, residual, ReLU; every element is read and written by one
// thread, so out may alias in or res.
template <int NT, int R>
__global__ void __launch_bounds__(NT) gn_reg_kernel(GnArgs a) {
    constexpr int NW = NT / 64;
    __shared__ double part[2][NW][256];
    __shared__ double chs[2][256];
    __shared__ float sc[256], sh[256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, C = a.C, L = a.L;
    const size_t b = blockIdx.x;
    const float4* in = (const float4*)(a.in + b * L * C);
    const int n4 = L * C / 4;
    float4 v[R];
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = in[min(tid + NT * u, n4 - 1)];
    // a thread's R values per channel summed in FP32, the rest of the
    // reduction in FP64
    float sf[4] = {0.f, 0.f, 0.f, 0.f}, qf[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < R; ++u) {
        if (tid + NT * u < n4) {
            const float e[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sf[k] += e[k];
                qf[k] = fmaf(e[k], e[k], qf[k]);
            }
        }
    }
    double s[4], q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        s[k] = sf[k];
        q[k] = qf[k];
    }
    // lane l holds channels 4l % C .. +3; lanes l and l xor m (m >= C/4) share them
    for (int off = C / 4; off < 64; off <<= 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s[k] += __shfl_xor(s[k], off);
            q[k] += __shfl_xor(q[k], off);
        }
    if (lane < C / 4)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            part[0][wv][4 * lane + k] = s[k];
            part[1][wv][4 * lane + k] = q[k];
        }
    __syncthreads();
    if (tid < C) {
        double cs = 0.0, cq = 0.0;
        for (int w = 0; w < NW; ++w) {
            cs += part[0][w][tid];
            cq += part[1][w][tid];
        }
        chs[0][tid] = cs;
        chs[1][tid] = cq;
    }
    __syncthreads();
    if (tid < C) {
        const int cpg = C / a.G, g = tid / cpg;
        double gs = 0.0, gq = 0.0;
        for (int c = g * cpg; c < (g + 1) * cpg; ++c) {
            gs += chs[0][c];
            gq += chs[1][c];
        }
        const double n = (double)cpg * L;
        const double mean = gs / n;
        const double var = fmax(gq / n - mean * mean, 0.0);
        const double scale = (double)a.gamma[tid] / sqrt(var + 1e-5);
        sc[tid] = (float)scale;
        sh[tid] = (float)((double)a.beta[tid] - mean * scale);
    }
    __syncthreads();
    const int c0 = (4 * tid) % C;
    const float4 S = make_float4(sc[c0], sc[c0 + 1], sc[c0 + 2], sc[c0 + 3]);
    const float4 H = make_float4(sh[c0], sh[c0 + 1], sh[c0 + 2], sh[c0 + 3]);
    float4* out = (float4*)(a.out + b * L * C);
    if (a.res) {
        // the residual in groups of RC float4s, to stay within 128 registers
        constexpr int RC = 4;
        const float4* res = (const float4*)(a.res + b * L * C);
#pragma unroll
        for (int u0 = 0; u0 < R; u0 += RC) {
            float4 r[RC];
#pragma unroll
            for (int u = 0; u < RC && u0 + u < R; ++u) r[u] = res[min(tid + NT * (u0 + u), n4 - 1)];
#pragma unroll
            for (int u = 0; u < RC && u0 + u < R; ++u) {
                float4& x = v[u0 + u];
                x = make_float4(fmaf(x.x, S.x, H.x) + r[u].x, fmaf(x.y, S.y, H.y) + r[u].y,
                                fmaf(x.z, S.z, H.z) + r[u].z, fmaf(x.w, S.w, H.w) + r[u].w);
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < R; ++u)
            v[u] = make_float4(fmaf(v[u].x, S.x, H.x), fmaf(v[u].y, S.y, H.y), fmaf(v[u].z, S.z, H.z),
                               fmaf(v[u].w, S.w, H.w));
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
        if (tid + NT * u < n4) {
            float4 y = v[u];
            if (a.relu) y = make_float4(fmaxf(y.x, 0.f), fmaxf(y.y, 0.f), fmaxf(y.z, 0.f), fmaxf(y.w, 0.f));
            out[tid + NT * u] = y;
        }
    }
}

}  // namespace afm
