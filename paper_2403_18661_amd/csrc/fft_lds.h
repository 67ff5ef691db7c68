// In-LDS complex FFT for one workgroup (Stockham autosort, radix 2/4/8/16),
// and the in-register DFTs (up to 32 points) that its passes are built from.
//
// The transform of length N = 2^LOGN lives in an LDS array of cpx<R>.  Every
// pass reads the elements of its butterflies into registers, waits at a
// barrier, and writes the results back to their autosorted positions, so a
// single LDS buffer suffices.  Pass with radix Rd and span Ns (product of the
// radices already applied), butterfly j < N/Rd:
//     v[r] = a[j + r N/Rd] * w^(r (j mod Ns)),  w = exp(-+2 pi i / (Ns Rd))
//     v    = DFT_Rd(v)
//     a[(j / Ns) Ns Rd + (j mod Ns) + r Ns] = v[r]
// Twiddles come from a table tw[t] = exp(-2 pi i t / N) built on the host in
// FP64; the inverse transform uses conjugates and is unnormalised.
// LDS addresses are padded by one element per 16 to spread bank accesses.
#pragma once
#include "common.h"

namespace afm {

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_padded_len(int n) { return n + (n >> 4); }

// cos(pi m / 16) for m = 0..8
__device__ __forceinline__ constexpr double cos_pi16(int m) {
    constexpr double C[9] = {1.0,
                             0.98078528040323044913,  // cos(pi/16)
                             0.92387953251128675613,  // cos(pi/8)
                             0.83146961230254523708,  // cos(3 pi/16)
                             0.70710678118654752440,  // cos(pi/4)
                             0.55557023301960222474,  // cos(5 pi/16)
                             0.38268343236508977173,  // cos(3 pi/8)
                             0.19509032201612826785,  // cos(7 pi/16)
                             0.0};
    m &= 31;  // one period is 32 steps of pi/16
    return m <= 8 ? C[m] : m <= 16 ? -C[16 - m] : m <= 24 ? -C[m - 16] : C[32 - m];
}

// exp(-2 pi i k / 32) (forward) or its conjugate (inverse), by symmetry from
// the cosines above; k is a compile-time constant wherever this is used.
template <typename R>
__device__ __forceinline__ cpx<R> w32(int k, bool inv) {
    const double c = cos_pi16(k);
    const double s = cos_pi16(k + 24);  // sin(x) = cos(x - pi/2)
    return {(R)c, (R)(inv ? s : -s)};
}

// In-register DFT of length RD (power of two <= 32) by radix-2 decimation in time.
template <typename R, int RD>
__device__ __forceinline__ void dft_reg(cpx<R>* v, bool inv) {
    if constexpr (RD == 1) {
        return;
    } else if constexpr (RD == 2) {
        cpx<R> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else {
        cpx<R> e[RD / 2], o[RD / 2];
#pragma unroll
        for (int i = 0; i < RD / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        dft_reg<R, RD / 2>(e, inv);
        dft_reg<R, RD / 2>(o, inv);
#pragma unroll
        for (int k = 0; k < RD / 2; ++k) {
            const int m = k * (32 / RD);  // twiddle exp(-+2 pi i m / 32)
            cpx<R> t;
            if (m == 0)
                t = o[k];
            else if (m == 8)  // times -i (forward) or +i (inverse): no multiplies
                t = inv ? cpx<R>{-o[k].y, o[k].x} : cpx<R>{o[k].y, -o[k].x};
            else
                t = cmul(o[k], w32<R>(m, inv));
            v[k] = cadd(e[k], t);
            v[k + RD / 2] = csub(e[k], t);
        }
    }
}

template <typename R, int LOGN, int NT, int RD, int NS>
__device__ __forceinline__ void fft_pass(cpx<R>* a, const cpx<R>* __restrict__ tw, bool inv) {
    constexpr int N = 1 << LOGN;
    constexpr int NB = N / RD;               // butterflies
    constexpr int PER = (NB + NT - 1) / NT;  // butterflies per thread
    cpx<R> v[PER][RD];
    const int tid = threadIdx.x;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = tid + p * NT;
        if (NB % NT == 0 || j < NB) {
            const int k = j % NS;
#pragma unroll
            for (int r = 0; r < RD; ++r) {
                cpx<R> x = a[lds_pad(j + r * NB)];
                if (NS > 1 && r > 0) {
                    cpx<R> w = tw[(r * k) * (N / (NS * RD))];
                    if (inv) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[p][r] = x;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = tid + p * NT;
        if (NB % NT == 0 || j < NB) {
            dft_reg<R, RD>(v[p], inv);
            const int base = (j / NS) * NS * RD + (j % NS);
#pragma unroll
            for (int r = 0; r < RD; ++r) a[lds_pad(base + r * NS)] = v[p][r];
        }
    }
    __syncthreads();
}

// Radix schedule: as many radix-16 passes as fit, then one smaller pass.
template <typename R, int LOGN, int NT, int NS = 1, int DONE = 0>
__device__ __forceinline__ void fft_passes(cpx<R>* a, const cpx<R>* __restrict__ tw, bool inv) {
    if constexpr (DONE < LOGN) {
        constexpr int LEFT = LOGN - DONE;
        constexpr int LR = LEFT >= 4 ? 4 : LEFT;
        constexpr int RD = 1 << LR;
        fft_pass<R, LOGN, NT, RD, NS>(a, tw, inv);
        fft_passes<R, LOGN, NT, NS * RD, DONE + LR>(a, tw, inv);
    }
}

// Full transform; the caller has written a[] (padded addresses) and synced.
template <typename R, int LOGN, int NT>
__device__ __forceinline__ void fft_lds(cpx<R>* a, const cpx<R>* __restrict__ tw, bool inv) {
    fft_passes<R, LOGN, NT>(a, tw, inv);
}

}  // namespace afm
