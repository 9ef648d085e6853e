// Batched power-of-two complex FFTs held in LDS (Stockham autosort).
//
// Forward transform X[m] = sum_j x[j] exp(-2 pi i j m / N).  NB transforms of
// length N live in LDS at buf[b * LD + j].  One radix-RAD Stockham stage with
// current span p (p = 1, RAD, RAD^2, ...) takes, for every j < N/RAD with
// k = j mod p, the inputs x[j + t N/RAD] (t < RAD), multiplies input t by
// exp(-2 pi i t k / (p RAD)), applies the length-RAD DFT and stores output q
// at (j - k) RAD + k + q p.  After all stages the result is in natural order.
// Every stage stages its inputs in registers, so a single LDS buffer suffices
// (barrier between the loads and the stores).  Twiddles come from a table
// tw[j] = exp(-2 pi i j / Nt) in global memory (cached), with Nt a multiple
// of N; `tws` = Nt / N.
#pragma once

#include "m2n_common.hpp"

namespace m2n {

template <typename R>
__device__ __forceinline__ void dft2(cplx<R>& a, cplx<R>& b) {
    cplx<R> s = cadd(a, b), d = csub(a, b);
    a = s;
    b = d;
}

// forward radix-4 butterfly on (u0,u1,u2,u3) in place, outputs in natural order
template <typename R>
__device__ __forceinline__ void dft4(cplx<R>* u) {
    cplx<R> a = cadd(u[0], u[2]), b = csub(u[0], u[2]);
    cplx<R> c = cadd(u[1], u[3]), d = csub(u[1], u[3]);
    u[0] = cadd(a, c);
    u[2] = csub(a, c);
    u[1] = {b.x + d.y, b.y - d.x};   // b - i d
    u[3] = {b.x - d.y, b.y + d.x};   // b + i d
}

// forward radix-8 butterfly in place, outputs in natural order: two
// length-4 DFTs of the even and odd inputs, combined with w8^q, w8 = e^{-i pi/4}
template <typename R>
__device__ __forceinline__ void dft8(cplx<R>* u) {
    cplx<R> e[4] = {u[0], u[2], u[4], u[6]};
    cplx<R> o[4] = {u[1], u[3], u[5], u[7]};
    dft4(e);
    dft4(o);
    const R h = (R)0.70710678118654752440;
    const cplx<R> o1 = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};    // w8 o1
    const cplx<R> o2 = {o[2].y, -o[2].x};                                 // -i o2
    const cplx<R> o3 = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};   // w8^3 o3
    u[0] = cadd(e[0], o[0]);
    u[4] = csub(e[0], o[0]);
    u[1] = cadd(e[1], o1);
    u[5] = csub(e[1], o1);
    u[2] = cadd(e[2], o2);
    u[6] = csub(e[2], o2);
    u[3] = cadd(e[3], o3);
    u[7] = csub(e[3], o3);
}

// Workgroup barrier for LDS traffic alone: waits for this wavefront's LDS
// operations (lgkmcnt), not for its global loads still in flight, so that a
// caller's prefetch of the next data stays in flight across the FFT (the
// stages exchange data only through LDS).  The memory clobber keeps the
// compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Position of element i of a transform in the padded layout of the
// intermediate stages: one free slot after every 2^psh elements (row length
// N + N / 2^psh).  A radix-8 stage with span p < 64 stores each butterfly's
// outputs 8 or 64 elements apart across lanes, which in the plain layout
// maps 32 lanes onto 4 or 8 of the 32 eight-byte bank pairs.  With psh = 3
// the lane strides become 9 and 72 (all 32 pairs for both stages); with
// psh = 5 (a shorter row) the first stage's stores are spread over all
// pairs and the second's over half of them.
__device__ __forceinline__ int fft_pad(int i, int psh) { return psh ? i + (i >> psh) : i; }

template <typename R, int N, int NB, int NT, int LD, int RAD, bool FIRST = false>
__device__ __forceinline__ void fft_stage(cplx<R>* buf, const cplx<R>* __restrict__ tw,
                                          int tws, int p, int nb, int in_psh = 0, int out_psh = 0) {
    constexpr int Q = N / RAD;              // butterflies per transform
    constexpr int BF = NB * Q;              // butterflies in the batch (at most)
    constexpr int IT = (BF + NT - 1) / NT;
    const int tid = threadIdx.x;
    const int bfr = nb * Q;                 // butterflies of the nb transforms present
    cplx<R> v[IT][RAD];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NT;
        if (idx < bfr) {
            const int b = idx / Q, j = idx - b * Q;
            const int k = j & (p - 1);
            const int tstep = k * (N / (p * RAD)) * tws;
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                cplx<R> val = buf[b * LD + fft_pad(j + t * Q, in_psh)];
                if (!FIRST && t > 0) val = cmul(val, tw[t * tstep]);   // first stage: k = 0
                v[it][t] = val;
            }
        }
    }
    lds_barrier();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NT;
        if (idx < bfr) {
            const int b = idx / Q, j = idx - b * Q;
            const int k = j & (p - 1);
            if constexpr (RAD == 8) dft8(v[it]);
            else if constexpr (RAD == 4) dft4(v[it]);
            else dft2(v[it][0], v[it][1]);
            const int base = (j - k) * RAD + k;
#pragma unroll
            for (int q = 0; q < RAD; ++q) buf[b * LD + fft_pad(base + q * p, out_psh)] = v[it][q];
        }
    }
    lds_barrier();
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// NB forward FFTs of length N (power of two, >= 2) in LDS: radix-8 stages
// while three or more factors of two remain, then one radix-4 or radix-2
// stage.  Caller must have synchronised after writing buf; returns
// synchronised.  With first_done (N >= 8) the caller has already stored the
// first radix-8 stage's output: when only x[0 .. N/8) can be non-zero, that
// output is x[j] repeated at positions 8 j .. 8 j + 7.  Only the first nb
// (<= NB) transforms are computed.  With PSH > 0 the stages between the
// first and the last use the padded layout (fft_pad; LD >= N + N / 2^PSH,
// and a first_done output is stored there); input and output are in the
// plain layout either way.
template <typename R, int N, int NB, int NT, int LD, int PSH = 0>
__device__ __forceinline__ void fft_lds(cplx<R>* buf, const cplx<R>* __restrict__ tw, int tws,
                                        bool first_done = false, int nb = NB) {
    constexpr int LOG = ilog2c(N);
    constexpr int N8 = LOG / 3, REM = LOG % 3;
    constexpr int NST = N8 + (REM ? 1 : 0);   // stages
    static_assert(PSH == 0 || LD >= N + (N >> PSH), "padded FFT rows need N + N / 2^PSH slots");
    constexpr int MID = NST > 1 ? PSH : 0;    // layout between stages
    int p = 1;
    if constexpr (N8 > 0) {
        if (!first_done) fft_stage<R, N, NB, NT, LD, 8, true>(buf, tw, tws, 1, nb, 0, MID);
        p = 8;
    }
#pragma unroll 1
    for (int s = 1; s < N8; ++s) {
        fft_stage<R, N, NB, NT, LD, 8>(buf, tw, tws, p, nb, MID, s + 1 < NST ? MID : 0);
        p *= 8;
    }
    if constexpr (REM == 2) fft_stage<R, N, NB, NT, LD, 4>(buf, tw, tws, p, nb, MID, 0);
    else if constexpr (REM == 1) fft_stage<R, N, NB, NT, LD, 2>(buf, tw, tws, p, nb, MID, 0);
}

}  // namespace m2n
