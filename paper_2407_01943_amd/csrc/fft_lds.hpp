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

// One stage with its span P and the layouts of its input and output known at
// compile time.  Reads x[j + t Q] sit at fixed distances from the padded
// position of j whenever Q is a whole number of padding blocks; writes
// base + q P likewise whenever P is a whole number of blocks or the RAD P
// outputs of a butterfly (an aligned run) fall in one block.  The offsets
// then fold into the LDS instructions instead of being computed per element.
// CIN (the second stage, P = 8): the input is the first stage's output for
// data confined to x[0 .. N/8), x[i / 8] at position i, read from the plain
// x[0 .. N/8) itself.
template <typename R, int N, int NB, int NT, int LD, int RAD, int P, int IN_PSH, int OUT_PSH, bool FIRST,
          bool CIN = false>
__device__ __forceinline__ void fft_stage(cplx<R>* buf, const cplx<R>* __restrict__ tw, int tws, int nb) {
    constexpr int Q = N / RAD;              // butterflies per transform
    constexpr int BF = NB * Q;              // butterflies in the batch (at most)
    constexpr int IT = (BF + NT - 1) / NT;
    static_assert(!CIN || (P == 8 && Q % 8 == 0), "compact input only for the second stage");
    constexpr bool RD_C = CIN || IN_PSH == 0 || Q % (1 << IN_PSH) == 0;
    constexpr int RD_STEP = CIN ? Q / 8 : Q + (IN_PSH ? Q >> IN_PSH : 0);
    constexpr bool WR_C = OUT_PSH == 0 || P % (1 << OUT_PSH) == 0 || (1 << OUT_PSH) % (P * RAD) == 0;
    constexpr int WR_STEP = P + (OUT_PSH && P >= (1 << OUT_PSH) ? P >> OUT_PSH : 0);
    const int tid = threadIdx.x;
    const int bfr = nb * Q;                 // butterflies of the nb transforms present
    cplx<R> v[IT][RAD];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NT;
        if (idx < bfr) {
            const int b = idx / Q, j = idx % Q;
            const int k = j & (P - 1);
            const int tstep = k * (N / (P * RAD)) * tws;
            const int rb = b * LD + (CIN ? j >> 3 : fft_pad(j, IN_PSH));
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                cplx<R> val = RD_C ? buf[rb + t * RD_STEP] : buf[b * LD + fft_pad(j + t * Q, IN_PSH)];
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
            const int b = idx / Q, j = idx % Q;
            const int k = j & (P - 1);
            if constexpr (RAD == 8) dft8(v[it]);
            else if constexpr (RAD == 4) dft4(v[it]);
            else dft2(v[it][0], v[it][1]);
            const int base = (j - k) * RAD + k;
            const int wb = b * LD + fft_pad(base, OUT_PSH);
#pragma unroll
            for (int q = 0; q < RAD; ++q) {
                if constexpr (WR_C) buf[wb + q * WR_STEP] = v[it][q];
                else buf[b * LD + fft_pad(base + q * P, OUT_PSH)] = v[it][q];
            }
        }
    }
    lds_barrier();
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// stages S .. NST - 1 of a length-N transform (span P at stage S): radix 8
// while three or more factors of two remain, then one radix-4 or radix-2
// stage; MID is the layout between stages
template <typename R, int N, int NB, int NT, int LD, int MID, int S, int NST, int P, bool CIN = false>
__device__ __forceinline__ void fft_stages(cplx<R>* buf, const cplx<R>* __restrict__ tw, int tws, int nb) {
    if constexpr (S < NST) {
        constexpr int LOG = ilog2c(N), N8 = LOG / 3, REM = LOG % 3;
        constexpr int RAD = S < N8 ? 8 : (REM == 2 ? 4 : 2);
        constexpr int IN = S > 0 && !CIN ? MID : 0;
        constexpr int OUT = S + 1 < NST ? MID : 0;
        fft_stage<R, N, NB, NT, LD, RAD, P, IN, OUT, S == 0, CIN>(buf, tw, tws, nb);
        fft_stages<R, N, NB, NT, LD, MID, S + 1, NST, P * RAD>(buf, tw, tws, nb);
    }
}

// NB forward FFTs of length N (power of two, >= 2) in LDS.  Caller must have
// synchronised after writing buf; returns synchronised.  With short_input
// (N >= 64) only x[0 .. N/8) can be non-zero and only those entries need be
// stored: the first radix-8 stage would just repeat x[j] at positions
// 8 j .. 8 j + 7, so the second stage reads x[0 .. N/8) directly.  Only the
// first nb (<= NB) transforms are computed.  With PSH > 0 the stages between
// the first and the last use the padded layout (fft_pad; LD >= N + N / 2^PSH);
// input and output are in the plain layout.
template <typename R, int N, int NB, int NT, int LD, int PSH = 0>
__device__ __forceinline__ void fft_lds(cplx<R>* buf, const cplx<R>* __restrict__ tw, int tws,
                                        bool short_input = false, int nb = NB) {
    constexpr int LOG = ilog2c(N);
    constexpr int N8 = LOG / 3, REM = LOG % 3;
    constexpr int NST = N8 + (REM ? 1 : 0);   // stages
    static_assert(PSH == 0 || LD >= N + (N >> PSH), "padded FFT rows need N + N / 2^PSH slots");
    constexpr int MID = NST > 1 ? PSH : 0;    // layout between stages
    if constexpr (N >= 64) {
        if (short_input) fft_stages<R, N, NB, NT, LD, MID, 1, NST, 8, true>(buf, tw, tws, nb);
        else fft_stages<R, N, NB, NT, LD, MID, 0, NST, 1>(buf, tw, tws, nb);
    } else {
        fft_stages<R, N, NB, NT, LD, MID, 0, NST, 1>(buf, tw, tws, nb);
    }
}

// forward radix-16 butterfly in place, outputs in natural order: four
// length-4 DFTs of the inputs n = 4 n1 + n2 (over n1), the twiddles
// w16^(n2 k1), then four length-4 DFTs over n2 (output k1 + 4 k2)
template <typename R>
__device__ __forceinline__ void dft16(cplx<R>* u) {
    const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173;
    const R h = (R)0.70710678118654752440;
    cplx<R> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        cplx<R> b[4] = {u[n2], u[4 + n2], u[8 + n2], u[12 + n2]};
        dft4(b);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = b[k1];
    }
    // w16^e = (cos(pi e / 8), -sin(pi e / 8)) for e = n2 k1
    y[1][1] = cmul(y[1][1], cplx<R>{c1, -s1});
    y[1][2] = cplx<R>{h * (y[1][2].x + y[1][2].y), h * (y[1][2].y - y[1][2].x)};
    y[1][3] = cmul(y[1][3], cplx<R>{s1, -c1});
    y[2][1] = cplx<R>{h * (y[2][1].x + y[2][1].y), h * (y[2][1].y - y[2][1].x)};
    y[2][2] = cplx<R>{y[2][2].y, -y[2][2].x};
    y[2][3] = cplx<R>{h * (y[2][3].y - y[2][3].x), -h * (y[2][3].x + y[2][3].y)};
    y[3][1] = cmul(y[3][1], cplx<R>{s1, -c1});
    y[3][2] = cplx<R>{h * (y[3][2].y - y[3][2].x), -h * (y[3][2].x + y[3][2].y)};
    y[3][3] = cmul(y[3][3], cplx<R>{-c1, s1});
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx<R> b[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        dft4(b);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) u[k1 + 4 * k2] = b[k2];
    }
}

// forward radix-32 butterfly in place: length-16 DFTs of the even and odd
// inputs, combined with w32^k = (cos(pi k / 16), -sin(pi k / 16))
template <typename R>
__device__ __forceinline__ void dft32(cplx<R>* u) {
    cplx<R> e[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        e[i] = u[2 * i];
        o[i] = u[2 * i + 1];
    }
    dft16(e);
    dft16(o);
    // cos(pi k / 16), k = 0 .. 8
    const R c[9] = {(R)1.0, (R)0.98078528040323044913, (R)0.92387953251128675613, (R)0.83146961230254523708,
                    (R)0.70710678118654752440, (R)0.55557023301960222474, (R)0.38268343236508977173,
                    (R)0.19509032201612826785, (R)0.0};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        // w32^k = cos(pi k / 16) - i sin(pi k / 16); sin(pi k / 16) = cos(pi (8 - k) / 16)
        const R cr = k <= 8 ? c[k] : -c[16 - k];
        const R si = k <= 8 ? c[8 - k] : c[k - 8];
        const cplx<R> t = k == 0 ? o[0] : cmul(o[k], cplx<R>{cr, -si});
        u[k] = cadd(e[k], t);
        u[k + 16] = csub(e[k], t);
    }
}

template <typename R, int RAD>
__device__ __forceinline__ void dft_r(cplx<R>* u) {
    if constexpr (RAD == 32) dft32(u);
    else if constexpr (RAD == 16) dft16(u);
    else if constexpr (RAD == 8) dft8(u);
    else if constexpr (RAD == 4) dft4(u);
    else dft2(u[0], u[1]);
}

// Orders a wavefront's LDS accesses without waiting for other wavefronts:
// a wavefront's LDS operations complete in issue order, so only the
// compiler has to be kept from moving them across this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wavefront-private transforms of length N = 64 E: one wavefront holds the
// whole transform, E values per lane, and exchanges them through its own LDS
// region (N + N / 2^PSH slots), so no workgroup barrier is involved.  Three
// Stockham stages: A (radix E, span 1, straight from the registers), B
// (radix RB, span E, E / RB butterflies per lane) and C (radix RC, span
// E RB, E / RC butterflies per lane); RB RC = 64.  The padding puts the
// stage-A stores (64 lanes E apart) and the stage-B stores on distinct
// banks.
template <int N>
struct WavePlan;
template <>
struct WavePlan<512> {
    static constexpr int E = 8, RB = 8, RC = 8, PSH = 3;
};
template <>
struct WavePlan<1024> {
    static constexpr int E = 16, RB = 16, RC = 4, PSH = 4;
};
template <>
struct WavePlan<2048> {
    static constexpr int E = 32, RB = 16, RC = 4, PSH = 5;
};

// Twiddle tables of a wavefront transform, tw = exp(-2 pi i j / N):
// stage B at twB[(t - 1) E + k] = tw[t k N / (E RB)] (t = 1 .. RB - 1,
// k < E) and stage C at twC[(t - 1) E RB + j] = tw[t j] (t = 1 .. RC - 1,
// j < E RB), so that a lane's twiddles for one t are consecutive across
// lanes.
template <int N>
struct WaveTw {
    static constexpr int E = WavePlan<N>::E, RB = WavePlan<N>::RB, RC = WavePlan<N>::RC;
    static constexpr int PC = E * RB;
    static constexpr int NB = (RB - 1) * E, NC = (RC - 1) * PC;
    // entry e of the combined table [twB, twC] as an index into tw
    __device__ static int index(int e) {
        if (e < NB) {
            const int t = e / E + 1, k = e % E;
            return t * k * (N / (E * RB));
        }
        const int e2 = e - NB, t = e2 / PC + 1, j = e2 % PC;
        return t * j;
    }
};

// Forward transform of one wavefront: lane l enters with x[l + 64 t] in
// v[t] (t < E) and leaves with X[l + 64 m] in v[m]; wb is the wavefront's
// LDS region, tw the combined table of WaveTw<N>.
template <typename R, int N>
__device__ __forceinline__ void wave_fft(cplx<R> (&v)[WavePlan<N>::E], cplx<R>* wb, const cplx<R>* tw) {
    using W = WavePlan<N>;
    constexpr int E = W::E, RB = W::RB, RC = W::RC, PSH = W::PSH;
    constexpr int PC = E * RB, SC = E / RC;
    const cplx<R>* twB = tw;
    const cplx<R>* twC = tw + WaveTw<N>::NB;
    const int l = threadIdx.x & 63;
    wave_lds_sync();   // the region's previous reads are done
    dft_r<R, E>(v);
#pragma unroll
    for (int q = 0; q < E; ++q) wb[fft_pad(l * E + q, PSH)] = v[q];
    wave_lds_sync();
    {
        // every butterfly's inputs are read before any output is stored
        constexpr int SB = E / RB, QB = N / RB;
        cplx<R> u[SB][RB];
#pragma unroll
        for (int s = 0; s < SB; ++s) {
            const int j = l + 64 * s, k = j & (E - 1);
#pragma unroll
            for (int t = 0; t < RB; ++t) {
                u[s][t] = wb[fft_pad(j + QB * t, PSH)];
                if (t > 0) u[s][t] = cmul(u[s][t], twB[(t - 1) * E + k]);
            }
        }
#pragma unroll
        for (int s = 0; s < SB; ++s) dft_r<R, RB>(u[s]);
        wave_lds_sync();
#pragma unroll
        for (int s = 0; s < SB; ++s) {
            const int j = l + 64 * s, k = j & (E - 1);
            const int base = (j - k) * RB + k;
#pragma unroll
            for (int q = 0; q < RB; ++q) wb[fft_pad(base + q * E, PSH)] = u[s][q];
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < SC; ++s) {
        const int j = l + 64 * s;
        cplx<R> u[RC];
#pragma unroll
        for (int t = 0; t < RC; ++t) {
            u[t] = wb[fft_pad(j + PC * t, PSH)];
            if (t > 0) u[t] = cmul(u[t], twC[(t - 1) * PC + j]);
        }
        dft_r<R, RC>(u);
#pragma unroll
        for (int q = 0; q < RC; ++q) v[s + SC * q] = u[q];
    }
}

}  // namespace m2n
