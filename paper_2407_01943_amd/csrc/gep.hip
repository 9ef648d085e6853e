// GPSS tapers at the nominal band (f_c0 = 0):  the K largest solutions of
//   R(A0) w = lambda R(B) w,   w^T R(B) w = 2 f_w              (Sec. 3.2, Sec. 2.2)
// with R(B)_{nm} = sin(2 pi f_max tau)/(pi tau), R(A0)_{nm} = sin(2 pi f_w tau)/(pi tau).
//
// Reduction: R(B) = L L^T (Cholesky), C = L^{-1} R(A0) L^{-T}, w = L^{-T} y with
// C y = lambda y.  The top-K eigenpairs of C come from block subspace
// iteration with Rayleigh-Ritz (block width p > K so the convergence factor
// lambda_{p+1} / lambda_K is tiny; the sinc spectrum plunges after about
// 2 f_w (t_N - t_1) eigenvalues).
//
// Two ways to apply C:
//  * lattice: every t_n is an integer and 2 f_max is a positive integer, so
//    every off-diagonal sin(2 pi f_max tau) vanishes and R(B) = 2 f_max I
//    exactly; R(A0) is Toeplitz in the lattice offset o_n = t_n - t_1 and
//    R(A0) v is a circular convolution on a zero-padded grid of M >= 2 S + 1
//    cells (S = o_N), evaluated with FP64 FFTs (two real columns packed into
//    one complex sequence).
//  * dense: R(B) and R(A0) are generated as FP64 matrices (padded to a
//    multiple of 64), R(B) is factored by a tiled right-looking Cholesky, and
//    C V = L^{-1} (R(A0) (L^{-T} V)) by blocked triangular solves and a GEMM.
// Everything is FP64.  The only host round trips are the residual norms read
// once per iteration and the Cholesky status.
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "fft_lds.hpp"
#include "m2n_common.hpp"

namespace m2n {

namespace {

constexpr int TB = 64;     // tile size of the dense path
constexpr int GNT = 256;   // threads per workgroup (general)
constexpr int GRAM_ROWS = 64;
constexpr int MAXP = 64;
constexpr int GRAM_WG_MAX = 128;   // workgroups of a Gram pass (partials reduced after)

// ------------------------------------------------------------ sinc kernel
// sin(pi u) with u first reduced to [-1/2, 1/2] by sin(pi (u - 2k)) = sin(pi u)
// and sin(pi (1 - r)) = sin(pi r); every step is exact, so integer u gives 0.
__device__ __forceinline__ double sinpi_red(double u) {
    double r = u - 2.0 * rint(0.5 * u);
    if (r > 0.5) r = 1.0 - r;
    else if (r < -0.5) r = -1.0 - r;
    return sinpi(r);
}

__device__ __forceinline__ double sinc_band(double f, double tau) {
    if (tau == 0.0) return 2.0 * f;
    return sinpi_red(2.0 * f * tau) / (M_PI * tau);
}

// cos(pi u) with u first reduced to [-1, 1] (exact)
__device__ __forceinline__ double cospi_red(double u) {
    return cospi(u - 2.0 * rint(0.5 * u));
}

// ----------------------------------------------------------- random start
__device__ __forceinline__ double hash_uniform(uint64_t key) {
    uint64_t z = key + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return ((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

__global__ void k_randinit(double* __restrict__ V, int64_t Np, int64_t N, int p, uint64_t seed) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (n >= Np || j >= p) return;
    V[(int64_t)j * Np + n] = n < N ? hash_uniform(seed * 0x100000001B3ull + (uint64_t)j * (uint64_t)Np + (uint64_t)n) : 0.0;
}

// ------------------------------------------------------ Gram matrices
// One pass over this workgroup's rows; the workgroup's partial sums of
//   [0 .. p*p)     V^T V   (entry i * p + j)
//   [p*p .. 2p*p)  V^T W   (nmat = 2)
// go to part + blockIdx.x * nmat * p * p; k_gram_reduce adds the partials
// in workgroup order, so the result does not depend on scheduling.
__global__ __launch_bounds__(GNT) void k_gram2(const double* __restrict__ V, const double* __restrict__ W,
                                               int64_t Np, int64_t nrows, int p, int nchunks_per_wg,
                                               int64_t nchunks, int nmat,
                                               double* __restrict__ part) {
    __shared__ double Vs[MAXP][GRAM_ROWS + 1];
    __shared__ double Ws[MAXP][GRAM_ROWS + 1];
    constexpr int PER = 2 * MAXP * MAXP / GNT;
    const int np = p * p;
    double acc[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) acc[e] = 0.0;
    const int64_t c0 = (int64_t)blockIdx.x * nchunks_per_wg;
    for (int64_t c = c0; c < c0 + nchunks_per_wg && c < nchunks; ++c) {
        const int64_t r0 = c * GRAM_ROWS;
        for (int e = threadIdx.x; e < p * GRAM_ROWS; e += GNT) {
            const int i = e / GRAM_ROWS, r = e % GRAM_ROWS;
            const bool in = r0 + r < nrows;
            Vs[i][r] = in ? V[(int64_t)i * Np + r0 + r] : 0.0;
            if (nmat > 1) Ws[i][r] = in ? W[(int64_t)i * Np + r0 + r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + e * GNT;
            if (idx < nmat * np) {
                const int which = idx >= np, q = idx - which * np;
                const int i = q / p, j = q % p;
                const double* b = which ? Ws[j] : Vs[j];
                double s = 0.0;
                for (int r = 0; r < GRAM_ROWS; ++r) s += Vs[i][r] * b[r];
                acc[e] += s;
            }
        }
        __syncthreads();
    }
    double* out = part + (int64_t)blockIdx.x * nmat * np;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = threadIdx.x + e * GNT;
        if (idx < nmat * np) out[idx] = acc[e];
    }
}

// One series of the low-rank GEP path.  Every low-rank kernel takes the
// descriptor by value for one series, or a device array indexed by
// blockIdx.y (blockIdx.x for the eigen-solver) for a batch.
struct LrSeries {
    const double* t;       // [N] sampling times
    const double* glx;     // Gauss-Legendre nodes [nq]; weights at glx + MAXP
    double* F;             // basis, column-major Np x pF
    double* gpart;         // Gram partials [nred][pF * pF]
    double* G;             // reduced Gram [pF * pF]
    double* Z;             // eigenvectors, Qn x K column-major
    double* theta;         // [K] eigenvalues (the lambda output on lattices)
    double* Y;             // expansion output (the tapers on lattices)
    int64_t N, Np, ldy;
    double tc, span, fw;
    double scale;          // eigen-solver input scale (1 / c)
    double wscale;         // fused taper scale sqrt(2 fw) / c
    double c;              // expansion scale without fusion
    int K, Qn, pF, nq, fuse, nchunks, cpw, nred;
};

__device__ __forceinline__ LrSeries lr_of(const LrSeries& d0, const LrSeries* D, int s) {
    return D ? D[s] : d0;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// Partial Gram matrix V^T V of this workgroup's rows on the FP64 matrix
// cores, one wavefront per workgroup.  V is column-major (leading dimension
// Np) with p <= 16 NT columns.  Each chunk of 64 rows is staged in LDS and
// fed to the 16x16x4 FP64 MFMA four rows at a time: lane l supplies
// A[i][k] = V[r_k][16 I + i] and B[k][j] = V[r_k][16 J + j] with
// i = j = l % 16, k = l / 16, and holds D[l / 16 + 4 v][l % 16] in
// accumulator element v (layout checked on the device).  Only the tiles I <= J are accumulated; the full
// symmetric p x p partial goes to part + blockIdx.x * p * p.
template <int NT>
__global__ __launch_bounds__(64) void k_gram_mfma(LrSeries d0, const LrSeries* D) {
    const LrSeries d = lr_of(d0, D, blockIdx.y);
    if ((int64_t)blockIdx.x * d.cpw >= d.nchunks) return;
    constexpr int NTT = NT * (NT + 1) / 2;
    __shared__ double Vs[16 * NT][GRAM_ROWS + 1];
    const int l = threadIdx.x;
    const int p = d.pF;
    const int64_t Np = d.Np;
    const double* __restrict__ V = d.F;
    d4 acc[NTT];
#pragma unroll
    for (int t = 0; t < NTT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t c0 = (int64_t)blockIdx.x * d.cpw;
    for (int64_t c = c0; c < c0 + d.cpw && c < d.nchunks; ++c) {
        const int64_t r0 = c * GRAM_ROWS;
        const bool inr = r0 + l < d.N;
        // unconditional loads from clamped addresses, so that all are in
        // flight together (rows < Np and columns < p are allocated)
        double ld[16 * NT];
#pragma unroll
        for (int i = 0; i < 16 * NT; ++i) ld[i] = V[(int64_t)(i < p ? i : p - 1) * Np + r0 + l];
#pragma unroll
        for (int i = 0; i < 16 * NT; ++i) Vs[i][l] = (i < p && inr) ? ld[i] : 0.0;
        __syncthreads();
#pragma unroll 4
        for (int ks = 0; ks < GRAM_ROWS / 4; ++ks) {
            const int r = 4 * ks + (l >> 4);
            double av[NT];
#pragma unroll
            for (int I = 0; I < NT; ++I) av[I] = Vs[16 * I + (l & 15)][r];
            int t = 0;
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int J = I; J < NT; ++J) {
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[I], av[J], acc[t], 0, 0, 0);
                    ++t;
                }
        }
        __syncthreads();
    }
    double* out = d.gpart + (int64_t)blockIdx.x * p * p;
    int t = 0;
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = I; J < NT; ++J) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + (l >> 4) + 4 * v, j = 16 * J + (l & 15);
                if (i < p && j < p) {
                    out[i * p + j] = acc[t][v];
                    if (I != J) out[j * p + i] = acc[t][v];
                }
            }
            ++t;
        }
}

// acc[i] = sum over the nwg partials of entry i, in a fixed order.  A
// workgroup takes 64 entries; its first NW wavefronts sum interleaved groups
// of U partials with all U loads in flight, then combine in LDS (the order
// depends only on NW, U and nwg; further wavefronts only join the barrier).
template <int NW, int U>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int nwg, int len,
                                             double* __restrict__ acc, int blk) {
    static_assert(NW == 4 || NW == 8, "four or eight wavefronts");
    __shared__ double red[NW][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blk * 64 + lane;
    const int ic = i < len ? i : len - 1;
    if (wv < NW) {
        double s[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] = 0.0;
        for (int g0 = U * wv; g0 < nwg; g0 += U * NW) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int g = g0 + u < nwg ? g0 + u : nwg - 1;
                v[u] = part[(int64_t)g * len + ic];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s[u % 8] += g0 + u < nwg ? v[u] : 0.0;
        }
        red[wv][lane] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    }
    __syncthreads();
    if (wv == 0 && i < len) {
        double t = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        if constexpr (NW == 8) t += (red[4][lane] + red[5][lane]) + (red[6][lane] + red[7][lane]);
        acc[i] = t;
    }
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int nwg, int len,
                                                      double* __restrict__ acc) {
    sum_partials<4, 8>(part, nwg, len, acc, blockIdx.x);
}

// the Gram matrix of each low-rank series from its partials; a series with
// more than 64 partials sums them on eight wavefronts with sixteen loads in
// flight each, otherwise on four with eight (the order depends only on the
// series' own partials, not on the rest of a batch)
__global__ __launch_bounds__(512) void k_gram_reduce(LrSeries d0, const LrSeries* D) {
    const LrSeries d = lr_of(d0, D, blockIdx.y);
    const int len = d.pF * d.pF;
    if ((int)blockIdx.x * 64 >= len) return;
    if (d.nred > 64) sum_partials<8, 16>(d.gpart, d.nred, len, d.G, blockIdx.x);
    else sum_partials<4, 8>(d.gpart, d.nred, len, d.G, blockIdx.x);
}

// ------------------------------------ top eigenpairs of a small symmetric
// move a double across lanes with a DPP pattern (both halves); lanes whose
// source is out of range or whose row is masked off receive 0
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over the 64 lanes, returned to every lane: quad permutes, row shifts
// and row broadcasts accumulate the total in lane 63, read back with
// readlane (cheaper than a ds_bpermute butterfly)
__device__ __forceinline__ double wsum(double v) {
    v += dpp_d<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp_d<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp_d<0x114, 0xf>(v);   // row_shr:4
    v += dpp_d<0x118, 0xf>(v);   // row_shr:8
    v += dpp_d<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// a double from lane l (l wave-uniform)
__device__ __forceinline__ double rdlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// a double moved across lanes by a DPP pattern; lanes without a source
// keep their own value (neutral for max and min)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_keep(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xf, false);
    const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xf, false);
    return __longlong_as_double(((long long)rhi << 32) | (unsigned int)rlo);
}

// max and min over the 64 lanes with the DPP pattern of wsum (every lane
// reaches lane 63 once), returned to every lane
__device__ __forceinline__ double wmax(double v) {
    v = fmax(v, dpp_keep<0xb1, 0xf>(v));
    v = fmax(v, dpp_keep<0x4e, 0xf>(v));
    v = fmax(v, dpp_keep<0x114, 0xf>(v));
    v = fmax(v, dpp_keep<0x118, 0xf>(v));
    v = fmax(v, dpp_keep<0x142, 0xa>(v));
    v = fmax(v, dpp_keep<0x143, 0xc>(v));
    return rdlane(v, 63);
}
__device__ __forceinline__ double wmin(double v) {
    v = fmin(v, dpp_keep<0xb1, 0xf>(v));
    v = fmin(v, dpp_keep<0x4e, 0xf>(v));
    v = fmin(v, dpp_keep<0x114, 0xf>(v));
    v = fmin(v, dpp_keep<0x118, 0xf>(v));
    v = fmin(v, dpp_keep<0x142, 0xa>(v));
    v = fmin(v, dpp_keep<0x143, 0xc>(v));
    return rdlane(v, 63);
}

// two independent wave sums, interleaved
__device__ __forceinline__ void wsum2(double (&v)[2]) {
#pragma unroll
    for (int u = 0; u < 2; ++u) v[u] += dpp_d<0xb1, 0xf>(v[u]);
#pragma unroll
    for (int u = 0; u < 2; ++u) v[u] += dpp_d<0x4e, 0xf>(v[u]);
#pragma unroll
    for (int u = 0; u < 2; ++u) v[u] += dpp_d<0x114, 0xf>(v[u]);
#pragma unroll
    for (int u = 0; u < 2; ++u) v[u] += dpp_d<0x118, 0xf>(v[u]);
#pragma unroll
    for (int u = 0; u < 2; ++u) v[u] += dpp_d<0x142, 0xa>(v[u]);
#pragma unroll
    for (int u = 0; u < 2; ++u) v[u] += dpp_d<0x143, 0xc>(v[u]);
#pragma unroll
    for (int u = 0; u < 2; ++u) v[u] = rdlane(v[u], 63);
}

// eight independent wave sums, interleaved so that the DPP steps of one
// hide the latency of the others
__device__ __forceinline__ void wsum8(double (&v)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += dpp_d<0xb1, 0xf>(v[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += dpp_d<0x4e, 0xf>(v[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += dpp_d<0x114, 0xf>(v[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += dpp_d<0x118, 0xf>(v[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += dpp_d<0x142, 0xa>(v[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += dpp_d<0x143, 0xc>(v[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = rdlane(v[u], 63);
}

// LDS of the small eigen-solver.  Row starts of Vh are 16-byte aligned so
// that a Lanczos vector is read as double2 pairs.
template <int LDA>
struct EigShared {
    double A[MAXP][LDA];         // input; then Sturm pairs, then LU rows
    double Vh[MAXP][MAXP + 2];   // Lanczos vector q_r in row r
    double X[MAXP][LDA];         // eigenvectors, X[k][i]
    double2 de[MAXP];            // (d_i, e_i) of the tridiagonal, e_{n-1} = 0
    double re[MAXP];             // 1 / e_i (0 where e_i = 0)
    double lam[MAXP];
    double tmp[2 * MAXP];
    double Gq[16 * MAXP];        // Gram and projection coefficients of a batch
};

// dot product of rows j and k of X over n components, eight at a time
template <int LDA>
__device__ __forceinline__ double xdot(const double (*X)[LDA], int j, int k, int n) {
    double s0 = 0.0, s1 = 0.0;
    for (int c0 = 0; c0 < n; c0 += 8) {
        double xa[8], xb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            xa[u] = c0 + u < n ? X[j][c0 + u] : 0.0;
            xb[u] = c0 + u < n ? X[k][c0 + u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            s0 += xa[u] * xb[u];
            s1 += xa[u + 1] * xb[u + 1];
        }
    }
    return s0 + s1;
}

// Orthonormalise the eigenvector batch X[kb..ke) (ke - kb <= 16) against
// the orthonormal X[0..kb) and among itself: block classical Gram-Schmidt
// followed by Cholesky QR, the pair applied `passes` times.  In exact
// arithmetic this is Gram-Schmidt in index order.
template <int LDA>
__device__ __forceinline__ void orth_batch(EigShared<LDA>& S, int n, int kb, int ke, int passes) {
    const int lane = threadIdx.x;
    const int nb = ke - kb;
    double* G = S.Gq;
    for (int pass = 0; pass < passes; ++pass) {
        if (kb > 0) {
            // C = X_prev^T X_batch (lane = coefficient), X_batch -= X_prev C
            for (int pr = lane; pr < kb * nb; pr += 64) G[pr] = xdot<LDA>(S.X, pr / nb, kb + pr % nb, n);
            __syncthreads();
            if (lane < n) {
                for (int k = kb; k < ke; ++k) {
                    double x = S.X[k][lane];
                    for (int j = 0; j < kb; ++j) x -= G[j * nb + (k - kb)] * S.X[j][lane];
                    S.X[k][lane] = x;
                }
            }
            __syncthreads();
        }
        // Gram matrix of the batch (upper triangle)
        for (int pr = lane; pr < nb * nb; pr += 64) {
            const int i = pr / nb, k = pr % nb;
            if (i <= k) G[pr] = xdot<LDA>(S.X, kb + i, kb + k, n);
        }
        __syncthreads();
        // G = R^T R in place (R upper), lane = column
        for (int j = 0; j < nb; ++j) {
            double s = 0.0;
            if (lane >= j && lane < nb) {
                s = G[j * nb + lane];
                for (int q = 0; q < j; ++q) s -= G[q * nb + j] * G[q * nb + lane];
            }
            const double rjj = sqrt(fmax(rdlane(s, j), 1e-280));
            if (lane >= j && lane < nb) G[j * nb + lane] = lane == j ? rjj : s / rjj;
            __syncthreads();
        }
        // X_batch <- X_batch R^{-1} (lane = component)
        if (lane < n) {
            double xs[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                xs[k] = 0.0;
                if (k < nb) {
                    double x = S.X[kb + k][lane];
#pragma unroll
                    for (int j = 0; j < k; ++j) x -= G[j * nb + k] * xs[j];
                    xs[k] = x / G[k * nb + k];
                }
            }
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < nb) S.X[kb + k][lane] = xs[k];
        }
        __syncthreads();
    }
}

// Numbers of eigenvalues of the tridiagonal below s0 and below s1: sign
// changes of p_i = (d_i - s) p_{i-1} - e_{i-1}^2 p_{i-2}, p_{-1} = 1,
// p_{-2} = 0, with exact power-of-two rescaling every four steps.  dq[i] =
// (d_i, e_{i-1}^2) for i < n4 (padding rows add no sign change).  Two
// chains per lane hide the latency of the recurrence; a sign change is the
// xor of consecutive sign bits.
template <int NP>
__device__ __forceinline__ void sturm_below2(const double2* dq, int n4, double s0, double s1,
                                             int& c0, int& c1) {
    double pp0 = 0.0, pc0 = 1.0, pp1 = 0.0, pc1 = 1.0;
    unsigned n0 = 0, n1 = 0, g0 = 0, g1 = 0;
#pragma unroll
    for (int j0 = 0; j0 < NP; j0 += 4) {
        if (j0 < n4) {
            double2 q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = dq[j0 + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double a0 = (q[u].x - s0) * pc0 - q[u].y * pp0;
                const double a1 = (q[u].x - s1) * pc1 - q[u].y * pp1;
                const unsigned h0 = (unsigned)__double2hiint(a0) >> 31;
                const unsigned h1 = (unsigned)__double2hiint(a1) >> 31;
                n0 += h0 ^ g0;
                n1 += h1 ^ g1;
                g0 = h0;
                g1 = h1;
                pp0 = pc0;
                pc0 = a0;
                pp1 = pc1;
                pc1 = a1;
            }
            const double m0 = fmax(fabs(pc0), fabs(pp0)), m1 = fmax(fabs(pc1), fabs(pp1));
            const double f0 = m0 > 0x1p+400 ? 0x1p-400 : (m0 < 0x1p-400 ? 0x1p+400 : 1.0);
            const double f1 = m1 > 0x1p+400 ? 0x1p-400 : (m1 < 0x1p-400 ? 0x1p+400 : 1.0);
            pc0 *= f0;
            pp0 *= f0;
            pc1 *= f1;
            pp1 *= f1;
        }
    }
    c0 = (int)n0;
    c1 = (int)n1;
}

// max of mx and min of mn over aligned groups of g lanes (g a power of two):
// quad permutes for partners 1 and 2, row shifts for 4 and 8 (the partner
// lies on one side or the other within the row), lane shuffles beyond
__device__ __forceinline__ void group_maxmin(double& mx, double& mn, int g) {
    const int lane = threadIdx.x;
    if (g > 1) {
        mx = fmax(mx, dpp_d<0xb1, 0xf>(mx));
        mn = fmin(mn, dpp_d<0xb1, 0xf>(mn));
    }
    if (g > 2) {
        mx = fmax(mx, dpp_d<0x4e, 0xf>(mx));
        mn = fmin(mn, dpp_d<0x4e, 0xf>(mn));
    }
    if (g > 4) {
        const bool up = (lane & 4) != 0;
        const double xa = dpp_d<0x104, 0xf>(mx), xb = dpp_d<0x114, 0xf>(mx);
        const double na = dpp_d<0x104, 0xf>(mn), nb = dpp_d<0x114, 0xf>(mn);
        mx = fmax(mx, up ? xb : xa);
        mn = fmin(mn, up ? nb : na);
    }
    if (g > 8) {
        const bool up = (lane & 8) != 0;
        const double xa = dpp_d<0x108, 0xf>(mx), xb = dpp_d<0x118, 0xf>(mx);
        const double na = dpp_d<0x108, 0xf>(mn), nb = dpp_d<0x118, 0xf>(mn);
        mx = fmax(mx, up ? xb : xa);
        mn = fmin(mn, up ? nb : na);
    }
    for (int o = 16; o < g; o <<= 1) {
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        mn = fmin(mn, __shfl_xor(mn, o, 64));
    }
}

// sweeps of inverse iteration: with shifts within a few ulps of |T| of the
// eigenvalues, two sweeps reduce the unwanted components below the
// eigenvectors' own condition unless two eigenvalues lie within about
// n^2 ulps of |T| of each other
constexpr int INVIT_SWEEPS = 2;

// 1/x from the hardware reciprocal and two Newton steps (|x| >= 1e-300)
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// deterministic start vector entry of inverse iteration, in [0.5, 1.5)
__device__ __forceinline__ double start_entry(int i, int k) {
    unsigned h = (unsigned)i * 0x9E3779B1u ^ ((unsigned)k + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return 0.5 + (double)(h >> 8) * (1.0 / 16777216.0);
}

// Top-K eigenpairs of a small symmetric matrix on one wavefront (64 lanes,
// n <= NP <= 64, NP a multiple of 8 sizing the per-lane register arrays).
// On entry S.A holds the matrix (row stride LDA); on exit S.lam[0..K)
// holds its K largest eigenvalues in descending order and S.X[k][0..n) the
// unit eigenvectors.
//  1. Lanczos with full re-orthogonalisation (two classical Gram-Schmidt
//     passes against every earlier vector): A Q_m = Q_m T_m + r e_m^T.  Lane
//     i keeps row i of A in registers; q_j goes to S.Vh[j].  The process
//     stops once |r| <= 1e-13 |A|_F with m >= K (the rounding noise of a
//     Gram matrix summed over 1e4..1e5 rows is about 1e-14 |A|), so T_m's
//     eigenvalues are eigenvalues of A to that accuracy; the spectra met
//     here (Gram matrices of band-limited bases) fall below it after about
//     2 f_w span + 10 values, so m is well below n (17 of 32 at 2 f_w span = 8).  If the Krylov space becomes invariant
//     before K vectors, the process continues from a new vector orthogonal
//     to it (T_m then splits into blocks).
//  2. Multisection on a division-free Sturm count of T_m: g lanes (a power
//     of two) bracket each wanted eigenvalue, and the next one, with two
//     samples each per round and combine the brackets by lane shuffles.
//  3. Eigenvectors of T_m (lane = eigenvector).  When the wanted
//     eigenvalues and the next one are at least 1e-8 |T| apart: twisted
//     factorisations of T_m - lam I and one Cholesky QR pass.  Otherwise
//     inverse iteration with partial-pivoting LU of T_m - lam I, each sweep
//     followed by orthonormalisation of the vectors in index order.
//     Rayleigh quotients give the final eigenvalues.
//  4. Ritz vectors X = Q_m Y (lane = component).
template <int LDA, int NP>
__device__ __forceinline__ void sym_topk_wave(EigShared<LDA>& S, int n_in, int K,
                                              long long* stamp = nullptr) {
    const int lane = threadIdx.x;
    const double eps = 2.220446049250313e-16;
    if (stamp && lane == 0) {
        stamp[0] = clock64();
        stamp[5] = 0;
        stamp[6] = 0;
    }
    // ---- 1. Lanczos with full re-orthogonalisation
    int m = n_in;
    {
        double a[NP];
        double fro = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            a[j] = (lane < n_in && j < n_in) ? S.A[lane][j] : 0.0;
            fro += a[j] * a[j];
        }
        // the Gram matrices this solver receives carry summation rounding of
        // about 1e-14 of their norm; a residual below 1e-13 |A|_F is noise
        const double btol = 1e-13 * sqrt(wsum(fro));
        double* wv = S.tmp;          // the vector being orthogonalised
        double* cf = S.tmp + MAXP;   // its coefficients on q_0 .. q_j
        // One classical Gram-Schmidt pass, w <- w - Q_{0..j} (Q_{0..j}^T w):
        // lane l forms q_l . w from LDS (rows of Vh not yet holding a Lanczos
        // vector are zero), then lane i subtracts its component, over the
        // rows 0..j in blocks of eight.  Every operand of a block is loaded
        // before the first product so that the LDS reads overlap.  Returns
        // the coefficient on q_j; `cc` receives this lane's coefficient
        // (lane l: on q_l, zero beyond j).
        auto cgs = [&](double& w, int j, double& cc) {
            wv[lane] = w;
            __syncthreads();
            const double2* qr = reinterpret_cast<const double2*>(S.Vh[lane < NP ? lane : 0]);
            const double2* wr = reinterpret_cast<const double2*>(wv);
            double2 x[NP / 2], y[NP / 2];
#pragma unroll
            for (int t = 0; t < NP / 2; ++t) {
                x[t] = qr[t];
                y[t] = wr[t];
            }
            __builtin_amdgcn_sched_barrier(0);
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
            for (int t = 0; t < NP / 2; t += 2) {
                s0 += x[t].x * y[t].x;
                s1 += x[t].y * y[t].y;
                s2 += x[t + 1].x * y[t + 1].x;
                s3 += x[t + 1].y * y[t + 1].y;
            }
            cc = lane < NP ? (s0 + s2) + (s1 + s3) : 0.0;
            cf[lane] = cc;
            __syncthreads();
            double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
            for (int l0 = 0; l0 <= j; l0 += 8) {
                double2 c[4];
                double v[8];
#pragma unroll
                for (int u = 0; u < 4; ++u) c[u] = *reinterpret_cast<const double2*>(cf + l0 + 2 * u);
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = S.Vh[l0 + u][lane];
                __builtin_amdgcn_sched_barrier(0);
                d0 += c[0].x * v[0];
                d1 += c[0].y * v[1];
                d2 += c[1].x * v[2];
                d3 += c[1].y * v[3];
                d0 += c[2].x * v[4];
                d1 += c[2].y * v[5];
                d2 += c[3].x * v[6];
                d3 += c[3].y * v[7];
            }
            w -= (d0 + d2) + (d1 + d3);
            const double cj = cf[j];
            __syncthreads();
            return cj;
        };
        for (int r = 0; r < NP; ++r) S.Vh[r][lane] = 0.0;
        double q = lane < n_in ? start_entry(lane, 777) : 0.0;
        q *= 1.0 / sqrt(wsum(q * q));
        double qprev = 0.0, bprev = 0.0;
        for (int j = 0; j < n_in; ++j) {
            S.Vh[j][lane] = q;
            __syncthreads();
            // w = A q_j, all of q_j loaded at once
            double2 u[NP / 2];
            const double2* qp = reinterpret_cast<const double2*>(S.Vh[j]);
#pragma unroll
            for (int t = 0; t < NP / 2; ++t) u[t] = qp[t];
            double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
            for (int t = 0; t < NP / 2; t += 2) {
                p0 += a[2 * t] * u[t].x;
                p1 += a[2 * t + 1] * u[t].y;
                p2 += a[2 * t + 2] * u[t + 1].x;
                p3 += a[2 * t + 3] * u[t + 1].y;
            }
            double w = lane < n_in ? (p0 + p2) + (p1 + p3) - bprev * qprev : 0.0;
            // three-term recurrence, then one re-orthogonalisation pass
            // against every earlier vector; a second pass only when the
            // first removed more than half of the norm (|w'|^2 < |c|^2, the
            // Daniel-Gragg-Kaufman-Stewart test), which keeps Q_m orthogonal
            // to rounding.  alpha_j accumulates every coefficient on q_j.
            double alpha = wsum(q * w);
            w -= alpha * q;
            double cc;
            alpha += cgs(w, j, cc);
            double s2[2] = {w * w, cc * cc};
            wsum2(s2);
            if (s2[0] < s2[1]) {
                alpha += cgs(w, j, cc);
                s2[0] = wsum(w * w);
            }
            const double beta = sqrt(s2[0]);
            if (lane == 0) S.de[j] = make_double2(alpha, 0.0);
            if (j + 1 == n_in) break;
            qprev = q;
            if (beta <= btol) {
                if (j + 1 >= K) {
                    m = j + 1;
                    break;
                }
                // invariant Krylov space: continue orthogonally to it
                w = lane < n_in ? start_entry(lane, 1000 + j) : 0.0;
                cgs(w, j, cc);
                cgs(w, j, cc);
                w *= 1.0 / sqrt(wsum(w * w));
                bprev = 0.0;
            } else {
                if (lane == 0) S.de[j].y = beta;
                w *= 1.0 / beta;
                bprev = beta;
            }
            q = w;
        }
        __syncthreads();
    }
    const int n = m;                   // order of the tridiagonal T_m
    const int n4 = (n + 3) & ~3;
    if (stamp && lane == 0) stamp[1] = clock64();
    // ---- 2. eigenvalues by multisection: the K wanted ones and, when T_m
    //         has it, the next one (its distance to the K-th decides the
    //         eigenvector method)
    const int Kb = K < n ? K + 1 : K;
    double glo = 1e300, ghi = -1e300;
    if (lane < n) {
        const double2 dl = S.de[lane];
        const double r = (lane > 0 ? fabs(S.de[lane - 1].y) : 0.0) + fabs(dl.y);
        glo = dl.x - r;
        ghi = dl.x + r;
        S.re[lane] = dl.y != 0.0 ? 1.0 / dl.y : 0.0;
    }
    glo = wmin(glo);
    ghi = wmax(ghi);
    const double tnorm = fmax(fmax(fabs(glo), fabs(ghi)), 1e-300);
    {
        double2* dq = reinterpret_cast<double2*>(&S.A[0][0]);
        if (lane < n4) {
            if (lane < n) {
                const double ep = lane > 0 ? S.de[lane - 1].y : 0.0;
                dq[lane] = make_double2(S.de[lane].x, lane > 0 ? fmax(ep * ep, 1e-200) : 0.0);
            } else {
                dq[lane] = make_double2(ghi + tnorm + 1.0, 0.0);
            }
        }
        __syncthreads();
        int g = 64;
        while (g > 1 && g * Kb > 64) g >>= 1;
        const int grp = lane / g, sub = lane - grp * g;
        const int idx = n - 1 - grp;
        const bool live = grp < Kb;
        const double tol = 1e-15 * tnorm;
        // invariant: count(l) <= idx < count(h)
        double l = glo - 2.0 * eps * tnorm, h = ghi + 2.0 * eps * tnorm;
        const double rsec = 1.0 / (double)(2 * g + 1);
        for (int round = 0; round < 200; ++round) {
            if (__all(!live || h - l <= tol)) break;
            const double st = (h - l) * rsec;
            const double s0 = l + (double)(2 * sub + 1) * st, s1 = l + (double)(2 * sub + 2) * st;
            int c0, c1;
            sturm_below2<NP>(dq, n4, s0, s1, c0, c1);
            double nl = l, nh = h;
            if (c0 > idx) nh = fmin(nh, s0);
            else nl = fmax(nl, s0);
            if (c1 > idx) nh = fmin(nh, s1);
            else nl = fmax(nl, s1);
            group_maxmin(nl, nh, g);
            if (h - l > tol) {
                l = nl;
                h = nh;
            }
        }
        if (live && sub == 0) S.lam[grp] = 0.5 * (l + h);
        __syncthreads();
    }
    if (stamp && lane == 0) stamp[2] = clock64();
    const double tiny = fmax(eps * tnorm, 1e-290);
    double mingap = 1e300;
    for (int k = 0; k + 1 < Kb; ++k) mingap = fmin(mingap, S.lam[k] - S.lam[k + 1]);
    if (mingap >= 1e-8 * tnorm) {
        // ---- 3a. separated eigenvalues: each eigenvector from a twisted
        //          factorisation of T - lam I (lane = eigenvector, batches of
        //          16).  With T - lam I = L D+ L^T = U D- U^T, the twist index
        //          r minimises |gamma_r| = |D+_r + D-_r - (d_r - lam)|, and
        //          z_r = 1, z_i = -(e_i / D+_i) z_{i+1} above r,
        //          z_i = -(e_{i-1} / D-_i) z_{i-1} below r, solves
        //          (T - lam I) z = gamma_r e_r.  Its error is that of one
        //          inverse-iteration step from the best unit start vector,
        //          rounding over the gap; one Cholesky QR pass restores
        //          orthonormality to rounding and normalises (z is stored
        //          unscaled).  Pivots that vanish are replaced by eps |T|.
        //          The bisection values are kept as the eigenvalues (within
        //          1e-15 |T|).
        double* Fp = &S.A[0][0];         // -e_i / D+_i
        double* Gm = Fp + 16 * MAXP;     // -e_{i-1} / D-_i
        double* Dp = Gm + 16 * MAXP;     // D+_i
        double* Dm = Dp + 16 * MAXP;     // D-_i
        for (int kb = 0; kb < K; kb += 16) {
            const int kk = kb + lane;
            const int kend = kb + 16 < K ? kb + 16 : K;
            long long ts0 = 0;
            if (stamp) ts0 = clock64();
            if (lane < 16 && kk < K) {
                const double lm = S.lam[kk];
                // forward (i) and backward (ib = n - 1 - i) pivots together,
                // the next step's tridiagonal entries fetched one step ahead
                double dp = S.de[0].x - lm, dm = S.de[n - 1].x - lm;
                double ea = S.de[0].y;
                double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
                if (n > 1) {
                    a = S.de[1];
                    b = S.de[n - 2];
                }
                Dp[lane] = dp;
                Dm[(n - 1) * 16 + lane] = dm;
                for (int i = 1; i < n; ++i) {
                    const int ib = n - 1 - i;
                    double2 a2 = make_double2(0.0, 0.0), b2 = make_double2(0.0, 0.0);
                    if (i + 1 < n) {
                        a2 = S.de[i + 1];
                        b2 = S.de[ib - 1];
                    }
                    const double rp = recip(dp != 0.0 ? dp : tiny);
                    const double rm = recip(dm != 0.0 ? dm : tiny);
                    Fp[(i - 1) * 16 + lane] = -ea * rp;
                    Gm[(ib + 1) * 16 + lane] = -b.y * rm;
                    dp = (a.x - lm) - ea * ea * rp;
                    dm = (b.x - lm) - b.y * b.y * rm;
                    Dp[i * 16 + lane] = dp;
                    Dm[ib * 16 + lane] = dm;
                    ea = a.y;
                    a = a2;
                    b = b2;
                }
                int r = 0;
                double gbest = 1e300;
#pragma unroll 4
                for (int i = 0; i < n; ++i) {
                    const double gi = fabs(Dp[i * 16 + lane] + Dm[i * 16 + lane] - (S.de[i].x - lm));
                    if (gi < gbest) {
                        gbest = gi;
                        r = i;
                    }
                }
                S.X[kk][r] = 1.0;
                double zu = 1.0, zd = 1.0;
#pragma unroll 4
                for (int st = 1; st < n; ++st) {
                    const int iu = r - st, id = r + st;
                    if (iu >= 0) {
                        zu *= Fp[iu * 16 + lane];
                        S.X[kk][iu] = zu;
                    }
                    if (id < n) {
                        zd *= Gm[id * 16 + lane];
                        S.X[kk][id] = zd;
                    }
                }
            }
            __syncthreads();
            long long ts1 = 0;
            if (stamp) ts1 = clock64();
            orth_batch(S, n, kb, kend, 1);
            if (stamp && lane == 0) {
                stamp[5] += ts1 - ts0;
                stamp[6] += clock64() - ts1;
            }
        }
    } else {
        // ---- 3b. eigenvalues within 1e-8 |T| of each other: inverse
        //         iteration in batches of 16 eigenvectors (lane =
        //         eigenvector); the LU rows of T - lam I live in A's storage,
        //         [i][lane], each pivot stored as its reciprocal
        double* U1 = &S.A[0][0];
        double* U2 = U1 + 16 * MAXP;
        double* U3 = U2 + 16 * MAXP;
        double* Bv = U3 + 16 * MAXP;
        for (int kb = 0; kb < K; kb += 16) {
            const int kk = kb + lane;
            const bool mine = lane < 16 && kk < K;
            const int kend = kb + 16 < K ? kb + 16 : K;
            if (mine)
                for (int i = 0; i < n; ++i) S.X[kk][i] = start_entry(i, kk);
            for (int it = 0; it < INVIT_SWEEPS; ++it) {
                long long ts0 = 0;
                if (stamp) ts0 = clock64();
                if (mine) {
                    double sh = S.lam[kk];
                    for (int j = 0; j < kk; ++j)
                        if (fabs(sh - S.lam[j]) < 10.0 * tiny) sh = S.lam[j] - 10.0 * tiny * (kk - j);
                    // forward elimination with partial pivoting, branch-free; the
                    // current row (c1, c2) and right-hand side cb are carried in
                    // registers and the next row's operands are fetched one step
                    // ahead
                    const double2 d0 = S.de[0];
                    double c1 = d0.x - sh, c2 = d0.y, sub = d0.y;
                    double cb = S.X[kk][0];
                    double2 nxt = n > 1 ? S.de[1] : make_double2(0.0, 0.0);
                    double rsub = S.re[0];
                    double nb = n > 1 ? S.X[kk][1] : 0.0;
                    for (int i = 0; i + 1 < n; ++i) {
                        double2 nxt2 = make_double2(0.0, 0.0);
                        double rsub2 = 0.0, nb2 = 0.0;
                        if (i + 2 < n) {
                            nxt2 = S.de[i + 2];
                            rsub2 = S.re[i + 1];
                            nb2 = S.X[kk][i + 2];
                        }
                        const double nd = nxt.x - sh, ne = nxt.y;
                        const bool swap = fabs(sub) > fabs(c1);
                        const double rp = recip(c1 != 0.0 ? c1 : tiny);
                        const double mult = swap ? c1 * rsub : sub * rp;
                        U1[i * 16 + lane] = swap ? rsub : rp;
                        U2[i * 16 + lane] = swap ? nd : c2;
                        U3[i * 16 + lane] = swap ? ne : 0.0;
                        Bv[i * 16 + lane] = swap ? nb : cb;
                        const double p1 = swap ? c2 : nd, q1 = swap ? nd : c2;
                        const double pb = swap ? cb : nb, qb = swap ? nb : cb;
                        c1 = p1 - mult * q1;
                        c2 = swap ? -mult * ne : ne;
                        cb = pb - mult * qb;
                        sub = ne;
                        nxt = nxt2;
                        rsub = rsub2;
                        nb = nb2;
                    }
                    const double rl = recip(c1 != 0.0 ? c1 : tiny);
                    // back substitution, the next row fetched one step ahead
                    double x1 = 0.0, x2 = 0.0;
                    double f1 = rl, f2 = 0.0, f3 = 0.0, fb = cb;
                    for (int i = n - 1; i >= 0; --i) {
                        double g1 = 0.0, g2 = 0.0, g3 = 0.0, gb = 0.0;
                        if (i > 0) {
                            g1 = U1[(i - 1) * 16 + lane];
                            g2 = U2[(i - 1) * 16 + lane];
                            g3 = U3[(i - 1) * 16 + lane];
                            gb = Bv[(i - 1) * 16 + lane];
                        }
                        const double v = (fb - f2 * x1 - f3 * x2) * f1;
                        S.X[kk][i] = v;
                        x2 = x1;
                        x1 = v;
                        f1 = g1;
                        f2 = g2;
                        f3 = g3;
                        fb = gb;
                    }
                }
                __syncthreads();
                long long ts1 = 0;
                if (stamp) ts1 = clock64();
                // one Cholesky QR pass between sweeps, two after the last
                orth_batch(S, n, kb, kend, it + 1 < INVIT_SWEEPS ? 1 : 2);
                if (stamp && lane == 0) {
                    stamp[5] += ts1 - ts0;
                    stamp[6] += clock64() - ts1;
                }
            }
        }
        // eigenvalue = Rayleigh quotient of the tridiagonal on the final
        // vector (the shifts of close eigenvalues were moved apart above)
        for (int k0 = 0; k0 < K; k0 += 8) {
            double s[8];
            const double2 dl = lane < n ? S.de[lane] : make_double2(0.0, 0.0);
            const double em = (lane > 0 && lane < n) ? S.de[lane - 1].y : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + u;
                double tx = 0.0, xi = 0.0;
                if (k < K && lane < n) {
                    xi = S.X[k][lane];
                    tx = dl.x * xi;
                    if (lane > 0) tx += em * S.X[k][lane - 1];
                    if (lane + 1 < n) tx += dl.y * S.X[k][lane + 1];
                }
                s[u] = xi * tx;
            }
            wsum8(s);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (lane == 0 && k0 + u < K) S.lam[k0 + u] = s[u];
        }
        __syncthreads();
    }
    if (stamp && lane == 0) stamp[3] = clock64();
    // ---- 4. Ritz vectors X = Q_m Y (lane = component), staged in A's storage
    {
        // Y padded with zeros to K4 = K rounded up to 4 rows and NP columns,
        // so that the product runs without branches
        double* XO = &S.A[0][0];
        const int K4 = (K + 3) & ~3;
        for (int k = 0; k < K4; ++k)
            if (lane < NP && (k >= K || lane >= n)) S.X[k][lane] = 0.0;
        __syncthreads();
        double qc[NP];
#pragma unroll
        for (int l = 0; l < NP; ++l) qc[l] = S.Vh[l][lane];   // rows >= n are zero
        for (int k0 = 0; k0 < K4; k0 += 4) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int l = 0; l < NP; ++l)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] += qc[l] * S.X[k0 + u][l];
#pragma unroll
            for (int u = 0; u < 4; ++u) XO[(k0 + u) * MAXP + lane] = acc[u];
        }
        __syncthreads();
        for (int k = 0; k < K; ++k)
            if (lane < n_in) S.X[k][lane] = XO[k * MAXP + lane];
        __syncthreads();
    }
    if (stamp && lane == 0) stamp[4] = clock64();
}

// K largest eigenpairs (theta_k, z_k) of the symmetric Qn x Qn leading
// block of scale * G (G row-major, leading dimension pF).  Output Z is
// column-major Qn x K (Z[i + k Qn] = component i of z_k), theta descending.
// With fuse != 0, rows Qn and Qn + 1 of G hold F^T 1 and F^T tau with
// tau_n = (tbar - t_n) / span, so that the two sign sums of the taper
// w_k = c_k F z_k are c_k (F^T 1) . z_k and c_k (F^T tau) . z_k: Z then
// receives +-wscale / sqrt(theta_k) z_k, the sign making the larger of the
// two sums positive.  One wavefront per series (blockIdx.x); Qn <= NP.
template <int NP>
__global__ __launch_bounds__(64) void k_sym_topk(LrSeries d0, const LrSeries* D, long long* stamp) {
    const LrSeries d = lr_of(d0, D, blockIdx.x);
    constexpr int LDA = MAXP + 1;
    __shared__ __align__(16) EigShared<LDA> S;
    const int lane = threadIdx.x;
    const int q = d.Qn, ld = d.pF, K = d.K;
    const double* __restrict__ G = d.G;
    for (int e_ = lane; e_ < q * q; e_ += 64) {
        const int i = e_ / q, j = e_ % q;
        S.A[i][j] = 0.5 * d.scale * (G[i * ld + j] + G[j * ld + i]);
    }
    __syncthreads();
    sym_topk_wave<LDA, NP>(S, q, K, stamp);
    if (d.fuse) {
        // sign sums, lane = taper
        if (lane < K) {
            double a = 0.0, b = 0.0;
            for (int i = 0; i < q; ++i) {
                const double z = S.X[lane][i];
                a += G[q * ld + i] * z;
                b += G[(q + 1) * ld + i] * z;
            }
            const double key = fabs(a) >= fabs(b) ? a : b;
            const double th = S.lam[lane];
            S.tmp[lane] = (key < 0.0 ? -d.wscale : d.wscale) / sqrt(th > 0.0 ? th : 1e-300);
        }
        __syncthreads();
        for (int e_ = lane; e_ < q * K; e_ += 64) {
            const int i = e_ % q, k = e_ / q;
            d.Z[e_] = S.tmp[k] * S.X[k][i];
        }
    } else {
        for (int e_ = lane; e_ < q * K; e_ += 64) {
            const int i = e_ % q, k = e_ / q;
            d.Z[e_] = S.X[k][i];
        }
    }
    if (lane < K) d.theta[lane] = S.lam[lane];
}

// register-array size picked from the largest matrix order of the launch
void launch_sym_topk(hipStream_t st, int maxq, int nseries, const LrSeries& d0, const LrSeries* D) {
    long long* ns = nullptr;
    const dim3 g((unsigned)nseries);
#define M2N_SYM(NPV) hipLaunchKernelGGL(k_sym_topk<NPV>, g, dim3(64), 0, st, d0, D, ns)
    if (maxq <= 16) M2N_SYM(16);
    else if (maxq <= 32) M2N_SYM(32);
    else if (maxq <= 40) M2N_SYM(40);
    else if (maxq <= 48) M2N_SYM(48);
    else M2N_SYM(64);
#undef M2N_SYM
}

// ------------------------------------- Rayleigh-Ritz on a general basis
// With G = V^T V = R^T R (Cholesky) and H = V^T W (W = C V), the Ritz pairs
// of C in span(V) are (theta, V Q) with Q = R^{-1} Q', where
// R^{-T} H R^{-1} = Q' diag(theta) Q'^T.  Y = V Q has orthonormal columns.
// Output: Q (column-major, Q[i + j p] = component i of Ritz vector j) and
// theta, in descending order of theta.  One wavefront.
template <int NP>
__global__ __launch_bounds__(64) void k_small_rr(double* __restrict__ acc, int p,
                                                 double* __restrict__ Qout,
                                                 double* __restrict__ theta) {
    constexpr int LDA = MAXP + 1;
    __shared__ double G[MAXP][LDA];     // V^T V, then R (upper)
    __shared__ __align__(16) EigShared<LDA> S;
    auto& H = S.A;                      // V^T W, then R^{-T} H R^{-1}
    const int tid = threadIdx.x;
    const int np = p * p;
    for (int e_ = tid; e_ < 2 * np; e_ += 64) {
        const double s = acc[e_];
        const int q = e_ % np, i = q / p, j = q % p;
        if (e_ < np) G[i][j] = s;
        else H[i][j] = s;
    }
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < p; ++i) dmax = fmax(dmax, G[i][i]);
    const double pfloor = dmax * 1e-24 + 1e-300;
    for (int j = 0; j < p; ++j) {
        if (tid == 0) {
            const double dd = G[j][j];
            G[j][j] = sqrt(dd > pfloor ? dd : pfloor);
        }
        __syncthreads();
        const double rjj = G[j][j];
        for (int c = j + 1 + tid; c < p; c += 64) G[j][c] /= rjj;
        __syncthreads();
        const int rem = p - j - 1;
        for (int e_ = tid; e_ < rem * rem; e_ += 64) {
            const int a = j + 1 + e_ / rem, b = j + 1 + e_ % rem;
            if (b >= a) G[a][b] -= G[j][a] * G[j][b];
        }
        __syncthreads();
    }
    for (int c = tid; c < p; c += 64) {   // H <- R^{-T} H
        for (int i = 0; i < p; ++i) {
            double s = H[i][c];
            for (int k = 0; k < i; ++k) s -= G[k][i] * H[k][c];
            H[i][c] = s / G[i][i];
        }
    }
    __syncthreads();
    for (int r = tid; r < p; r += 64) {   // H <- H R^{-1}
        for (int j = 0; j < p; ++j) {
            double s = H[r][j];
            for (int k = 0; k < j; ++k) s -= H[r][k] * G[k][j];
            H[r][j] = s / G[j][j];
        }
    }
    __syncthreads();
    for (int e_ = tid; e_ < np; e_ += 64) {
        const int i = e_ / p, j = e_ % p;
        if (i < j) {
            const double m = 0.5 * (H[i][j] + H[j][i]);
            H[i][j] = m;
            H[j][i] = m;
        }
    }
    __syncthreads();
    sym_topk_wave<LDA, NP>(S, p, p);
    for (int jc = tid; jc < p; jc += 64) {   // Q = R^{-1} Q'
        for (int i = p - 1; i >= 0; --i) {
            double s = S.X[jc][i];
            for (int k = i + 1; k < p; ++k) s -= G[i][k] * Qout[k + jc * p];
            Qout[i + jc * p] = s / G[i][i];
        }
        theta[jc] = S.lam[jc];
    }
}

// ------------------------------------------- quadrature basis of R(A0)
// R(A0)_{nm} = int_{-fw}^{fw} e^{j 2 pi f (t_n - t_m)} df.  With Gauss-Legendre
// nodes +-f_q = +-fw x_q and weights fw g_q on [-fw, fw] (symmetric pairs),
// the imaginary parts cancel and R(A0) = F F^T with 2 columns per positive
// node
//   F[2q][n] = sqrt(2 fw g_q) cos(2 pi f_q tau_n),
//   F[2q+1][n] = sqrt(2 fw g_q) sin(2 pi f_q tau_n),   tau_n = t_n - t_c.
// With aux != 0 two more columns hold 1 and (t_c - t_n) / span, whose
// products with F give the sign sums of the tapers.  Rows n >= N are zero.
// Column-major with leading dimension Np; grid (Np / 256, nq + aux).
// one sample per thread, LR_QB quadrature nodes per workgroup row
// (blockIdx.y); the auxiliary columns go with the last row; padding rows zero
constexpr int LR_QB = 4;
__global__ __launch_bounds__(256) void k_lr_basis(LrSeries d0, const LrSeries* D) {
    const LrSeries d = lr_of(d0, D, blockIdx.z);
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q0 = (int)blockIdx.y * LR_QB;
    if (n >= d.Np || q0 >= d.nq + (d.pF > d.Qn ? 1 : 0)) return;
    const bool live = n < d.N;
    const double tn = live ? d.t[n] : d.tc;
    const int q1 = q0 + LR_QB < d.nq ? q0 + LR_QB : d.nq;
    for (int q = q0; q < q1; ++q) {
        double c = 0.0, s = 0.0;
        if (live) {
            sincospi(2.0 * d.fw * d.glx[q] * (tn - d.tc), &s, &c);
            const double sq = sqrt(2.0 * d.fw * d.glx[MAXP + q]);
            c *= sq;
            s *= sq;
        }
        d.F[(int64_t)(2 * q) * d.Np + n] = c;
        d.F[(int64_t)(2 * q + 1) * d.Np + n] = s;
    }
    if (d.pF > d.Qn && q0 + LR_QB > d.nq) {
        d.F[(int64_t)(2 * d.nq) * d.Np + n] = live ? 1.0 : 0.0;
        d.F[(int64_t)(2 * d.nq + 1) * d.Np + n] = live ? (d.tc - tn) / d.span : 0.0;
    }
}

// Y[k * ldy + n] = s_k * sum_j F[j][n] Z[j + k Qn] for k < K, n < ldy, with
// s_k = 1 / sqrt(c theta_k), or 1 when the eigen-solver already scaled Z
template <int QC>
__global__ __launch_bounds__(64) void k_lr_expand(LrSeries d0, const LrSeries* D) {
    const LrSeries d = lr_of(d0, D, blockIdx.y);
    const int64_t n = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if ((int64_t)blockIdx.x * 64 >= d.ldy) return;
    __shared__ double Zs[QC * MAXP];
    __shared__ double sk[MAXP];
    const int q = d.Qn, K = d.K;
    for (int e = threadIdx.x; e < QC * K; e += 64) {
        const int j = e % QC, k = e / QC;
        Zs[e] = j < q ? d.Z[j + k * q] : 0.0;
    }
    for (int k = threadIdx.x; k < K; k += 64) sk[k] = d.fuse ? 1.0 : 1.0 / sqrt(d.c * d.theta[k]);
    __syncthreads();
    if (n >= d.ldy) return;
    // unconditional loads from clamped addresses (rows < Np and columns < q
    // are allocated), so that all are in flight together
    double a[QC];
#pragma unroll
    for (int j = 0; j < QC; ++j) a[j] = d.F[(int64_t)(j < q ? j : q - 1) * d.Np + n];
#pragma unroll
    for (int j = 0; j < QC; ++j) a[j] = (j < q && n < d.N) ? a[j] : 0.0;
    for (int k = 0; k < K; ++k) {
        double y = 0.0;
#pragma unroll
        for (int j = 0; j < QC; ++j) y += a[j] * Zs[k * QC + j];
        d.Y[(int64_t)k * d.ldy + n] = y * sk[k];
    }
}

// ------------------------------------- checks of the sampling times
// Per workgroup: flags (bit 0 a non-finite t_n, bit 1 a step t_n <= t_{n-1},
// bit 2 a t_n that is not an integer of magnitude <= 4e15) and the first
// offending indices; workgroup 0 also stores t_0 and t_{N-1}.  The record
// lives in pinned host memory and is read after the stream synchronises.
struct TInfo {
    int flags;
    int pad;
    unsigned long long first_nonfinite, first_order;
};

// one series of a t check: ranges of per_wg samples, records at info / hdr
struct TaSeries {
    const double* t;
    int64_t N, per_wg;
    int nblk, pad;
    TInfo* info;      // [nblk]
    double* hdr;      // [2]
};

__global__ __launch_bounds__(256) void k_t_analyze(TaSeries d0, const TaSeries* D) {
    const TaSeries d = D ? D[blockIdx.y] : d0;
    if ((int)blockIdx.x >= d.nblk) return;
    __shared__ int sf;
    __shared__ unsigned long long snf, sord;
    if (threadIdx.x == 0) {
        sf = 0;
        snf = ~0ull;
        sord = ~0ull;
    }
    __syncthreads();
    const double* __restrict__ t = d.t;
    const int64_t N = d.N;
    const int64_t b0 = (int64_t)blockIdx.x * d.per_wg;
    const int64_t b1 = b0 + d.per_wg < N ? b0 + d.per_wg : N;
    int flags = 0;
    unsigned long long fnf = ~0ull, ford = ~0ull;
    for (int64_t n = b0 + threadIdx.x; n < b1; n += 256) {
        const double v = t[n];
        if (!isfinite(v)) {
            flags |= 1;
            fnf = fnf < (unsigned long long)n ? fnf : (unsigned long long)n;
            continue;
        }
        if (n > 0 && !(v > t[n - 1])) {
            flags |= 2;
            ford = ford < (unsigned long long)n ? ford : (unsigned long long)n;
        }
        if (v != rint(v) || fabs(v) > 4.0e15) flags |= 4;
    }
    if (flags) atomicOr(&sf, flags);
    if (fnf != ~0ull) atomicMin(&snf, fnf);
    if (ford != ~0ull) atomicMin(&sord, ford);
    __syncthreads();
    if (threadIdx.x == 0) {
        d.info[blockIdx.x].flags = sf;
        d.info[blockIdx.x].first_nonfinite = snf;
        d.info[blockIdx.x].first_order = sord;
        if (blockIdx.x == 0) {
            d.hdr[0] = t[0];
            d.hdr[1] = t[N - 1];
        }
    }
}

// ---------------------------------- Ritz vectors, next block, residuals
// Y = V Q (orthonormal Ritz vectors), Z = W Q = C Y;
//   res[wg][k] = sum_n (Z_nk - theta_k Y_nk)^2        (k < K)
//   V <- Z diag(1 / max(theta, floor))  (next block; in place)
// Rows >= N are zero.  PC is p rounded up to a multiple of 8; one row per
// thread, 64 threads per workgroup.
template <int PC>
__global__ __launch_bounds__(64) void k_rotate2(double* __restrict__ V, const double* __restrict__ W,
                                                const double* __restrict__ Q,
                                                const double* __restrict__ theta, int64_t Np,
                                                int64_t N, int p, int K, double* __restrict__ Y,
                                                double* __restrict__ res) {
    __shared__ double Qs[PC * PC];
    __shared__ double th[PC];
    for (int e = threadIdx.x; e < PC * PC; e += 64) {
        const int i = e % PC, j = e / PC;
        Qs[e] = (i < p && j < p) ? Q[i + j * p] : 0.0;
    }
    for (int e = threadIdx.x; e < PC; e += 64) th[e] = e < p ? theta[e] : 1.0;
    __syncthreads();
    const double floor_t = fabs(th[0]) * 1e-6 + 1e-300;
    const int64_t n = (int64_t)blockIdx.x * 64 + threadIdx.x;
    double rk[PC];
#pragma unroll
    for (int j = 0; j < PC; ++j) rk[j] = 0.0;
    if (n < N) {
        double vr[PC], wr[PC];
#pragma unroll
        for (int i = 0; i < PC; ++i) {
            vr[i] = i < p ? V[(int64_t)i * Np + n] : 0.0;
            wr[i] = i < p ? W[(int64_t)i * Np + n] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < PC; ++j) {
            if (j < p) {
                double y = 0.0, z = 0.0;
#pragma unroll
                for (int i = 0; i < PC; ++i) {
                    const double q = Qs[j * PC + i];
                    y += vr[i] * q;
                    z += wr[i] * q;
                }
                Y[(int64_t)j * Np + n] = y;
                const double tj = th[j];
                V[(int64_t)j * Np + n] = z / (tj > floor_t ? tj : floor_t);
                const double d = z - tj * y;
                rk[j] = d * d;
            }
        }
    } else if (n < Np) {
        for (int j = 0; j < p; ++j) {
            Y[(int64_t)j * Np + n] = 0.0;
            V[(int64_t)j * Np + n] = 0.0;
        }
    }
    // all 64 lanes are active here
#pragma unroll
    for (int j = 0; j < PC; ++j) {
        if (j < K) {
            double v = rk[j];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (threadIdx.x == 0) res[(int64_t)blockIdx.x * K + j] = v;
        }
    }
}

// ------------------------------------------------------ lattice helpers
__global__ void k_fill_int(int* __restrict__ a, int64_t n, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// map[t_n - t_0] = n for integer sampling times
__global__ void k_lattice_map(const double* __restrict__ t, int64_t N, int* __restrict__ map) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) map[(int64_t)(t[n] - t[0])] = (int)n;
}

// h[l] = s(l) for l <= S, s(l - M) for l >= M - S, else 0 (complex, imag 0)
__global__ void k_toep_kernel(cplx<double>* __restrict__ h, int64_t M, int64_t S, double f) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= M) return;
    double v = 0.0;
    if (l <= S) v = sinc_band(f, (double)l);
    else if (l >= M - S) v = sinc_band(f, (double)(l - M));
    h[l] = {v, 0.0};
}

// Hhat[m] = Re(F[m]) * scale
__global__ void k_real_scale(const cplx<double>* __restrict__ F, int64_t M, double scale,
                             double* __restrict__ out) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) out[m] = F[m].x * scale;
}

// ------------------------------------------- FP64 FFTs for the convolution
// Source modes for the first pass / whole transform:
//   SRC_DIRECT: src[b * M + l]
//   SRC_PAIR:   V[2b][map[l]] + i V[2b+1][map[l]] (0 where map = -1)
// Destination modes:
//   DST_DIRECT: dst[b * M + m] = F[m]
//   DST_MULCONJ: dst[b * M + m] = Hhat[m] * conj(F[m])
//   DST_PAIR:   Y[2b][map[m]] = Re F[m], Y[2b+1][map[m]] = -Im F[m]
enum { SRC_DIRECT = 0, SRC_PAIR = 1 };
enum { DST_DIRECT = 0, DST_MULCONJ = 1, DST_PAIR = 2 };

struct ConvArgs {
    const cplx<double>* src;
    const double* V;
    const int* map;
    int64_t Np;
    int p;
    cplx<double>* dst;
    const double* Hhat;
    double* Y;
};

__device__ __forceinline__ cplx<double> conv_load(const ConvArgs& a, int mode, int b, int64_t M,
                                                   int64_t l) {
    if (mode == SRC_DIRECT) return a.src[(int64_t)b * M + l];
    const int n = a.map[l];
    if (n < 0) return {0.0, 0.0};
    const int j0 = 2 * b, j1 = 2 * b + 1;
    const double re = a.V[(int64_t)j0 * a.Np + n];
    const double im = j1 < a.p ? a.V[(int64_t)j1 * a.Np + n] : 0.0;
    return {re, im};
}

__device__ __forceinline__ void conv_store(const ConvArgs& a, int mode, int b, int64_t M, int64_t m,
                                           cplx<double> F) {
    if (mode == DST_DIRECT) {
        a.dst[(int64_t)b * M + m] = F;
    } else if (mode == DST_MULCONJ) {
        const double hh = a.Hhat[m];
        a.dst[(int64_t)b * M + m] = {hh * F.x, -hh * F.y};
    } else {
        const int n = a.map[m];
        if (n < 0) return;
        const int j0 = 2 * b, j1 = 2 * b + 1;
        a.Y[(int64_t)j0 * a.Np + n] = F.x;
        if (j1 < a.p) a.Y[(int64_t)j1 * a.Np + n] = -F.y;
    }
}

// whole transform in one workgroup (M <= 4096)
template <int MS>
__global__ __launch_bounds__(GNT) void k_fft_small(ConvArgs a, int smode, int dmode,
                                                   const cplx<double>* __restrict__ tw) {
    __shared__ cplx<double> buf[MS];
    const int b = blockIdx.x;
    for (int l = threadIdx.x; l < MS; l += GNT) buf[l] = conv_load(a, smode, b, MS, l);
    __syncthreads();
    fft_lds<double, MS, 1, GNT, MS>(buf, tw, 1);
    for (int m = threadIdx.x; m < MS; m += GNT) conv_store(a, dmode, b, MS, m, buf[m]);
}

// two-pass transform, pass A: columns l2 in [a0, a0 + BB), FFT over l1, twiddle
template <int N1, int BB>
__global__ __launch_bounds__(GNT) void k_fftA(ConvArgs a, int smode, int log_N2, int64_t M,
                                              const cplx<double>* __restrict__ tw, int tws,
                                              const cplx<double>* __restrict__ tw_lo,
                                              const cplx<double>* __restrict__ tw_hi, int lo_bits,
                                              cplx<double>* __restrict__ inter) {
    constexpr int LD = N1 + 1;
    __shared__ cplx<double> tile[BB * LD];
    const int N2 = 1 << log_N2;
    const int nblk = N2 / BB;
    const int blk = blockIdx.x % nblk;
    const int b = blockIdx.x / nblk;
    const int a0 = blk * BB;
    for (int e = threadIdx.x; e < BB * N1; e += GNT) {
        const int cb = e % BB, l1 = e / BB;
        tile[cb * LD + l1] = conv_load(a, smode, b, M, (int64_t)(a0 + cb) + ((int64_t)l1 << log_N2));
    }
    __syncthreads();
    fft_lds<double, N1, BB, GNT, LD>(tile, tw, tws);
    const int lo_mask = (1 << lo_bits) - 1;
    for (int e = threadIdx.x; e < BB * N1; e += GNT) {
        const int cb = e % BB, m1 = e / BB;
        const int q = (a0 + cb) * m1;
        const cplx<double> twv = cmul(tw_lo[q & lo_mask], tw_hi[q >> lo_bits]);
        inter[(int64_t)b * M + (int64_t)m1 * N2 + a0 + cb] = cmul(tile[cb * LD + m1], twv);
    }
}

// pass B: rows m1 in [r0, r0 + MM), FFT over l2, output m = m1 + N1 m2
template <int N2, int MM>
__global__ __launch_bounds__(GNT) void k_fftB(ConvArgs a, int dmode, int N1, int64_t M,
                                              const cplx<double>* __restrict__ inter,
                                              const cplx<double>* __restrict__ tw, int tws) {
    constexpr int LD = N2 + 1;
    __shared__ cplx<double> rows[MM * LD];
    const int nrb = N1 / MM;
    const int rb = blockIdx.x % nrb;
    const int b = blockIdx.x / nrb;
    const int r0 = rb * MM;
    const cplx<double>* src = inter + (int64_t)b * M + (int64_t)r0 * N2;
    for (int e = threadIdx.x; e < MM * N2; e += GNT) {
        const int mm = e / N2, l2 = e % N2;
        rows[mm * LD + l2] = src[(int64_t)mm * N2 + l2];
    }
    __syncthreads();
    fft_lds<double, N2, MM, GNT, LD>(rows, tw, tws);
    for (int e = threadIdx.x; e < MM * N2; e += GNT) {
        const int mm = e % MM, m2 = e / MM;
        conv_store(a, dmode, b, M, (int64_t)(r0 + mm) + (int64_t)N1 * m2, rows[mm * LD + m2]);
    }
}

// ------------------------------------------------------------ dense path
// R[i + j Np] = s(t_i - t_j) for i, j < N; padding: diag = pad_diag, else 0
__global__ void k_gen_sinc(const double* __restrict__ t, int64_t N, int64_t Np, double f,
                           double pad_diag, double* __restrict__ R) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= Np) return;
    double v;
    if (i < N && j < N) v = sinc_band(f, t[i] - t[j]);
    else v = (i == j) ? pad_diag : 0.0;
    R[i + j * Np] = v;
}

// R[i + j Np] = R(B^q)(t_i - t_j) of the sub-band f_min <= |f| <= f_max
// (Sec. 2.4): 2 cos(pi (f_max + f_min) tau) sin(pi (f_max - f_min) tau) / (pi tau),
// diagonal 2 (f_max - f_min); padding: diag 1, else 0
__global__ void k_gen_subband(const double* __restrict__ t, int64_t N, int64_t Np, double fmin,
                              double fmax, double* __restrict__ R) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= Np) return;
    double v;
    if (i < N && j < N) {
        const double tau = t[i] - t[j];
        v = tau == 0.0 ? 2.0 * (fmax - fmin)
                       : 2.0 * cospi_red((fmax + fmin) * tau) * sinpi_red((fmax - fmin) * tau) / (M_PI * tau);
    } else {
        v = (i == j) ? 1.0 : 0.0;
    }
    R[i + j * Np] = v;
}

// Cholesky of the TB x TB diagonal block kb in place (lower; upper zeroed).
// Four wavefronts; lane i of wavefront q holds columns 16q .. 16q + 15 of row
// i in registers.  At column j the owning wavefront takes the pivot (lane j's
// element), scales the column and stages it in LDS; after one barrier every
// lane updates its columns k > j from its own element l_ij and broadcast
// reads of l_kj.  A pivot <= 0 records the first failing row in status and
// the factorisation continues with 1 so that every launch completes.
__global__ __launch_bounds__(TB * 4) void k_potrf(double* __restrict__ A, int64_t Np, int kb, int64_t N,
                                                  int* __restrict__ status) {
    constexpr int CW = TB / 4;   // columns per wavefront
    __shared__ double col[2][TB];
    const int i = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t o = (int64_t)kb * TB;
    double r[CW];
#pragma unroll
    for (int u = 0; u < CW; ++u) r[u] = A[(o + i) + (o + CW * q + u) * Np];
    // column j = CW qq + u with u unrolled, so that the owner's pivot column
    // is a register of static index (no select chains over r)
#pragma unroll 1
    for (int qq = 0; qq < 4; ++qq) {
#pragma unroll
        for (int u = 0; u < CW; ++u) {
            const int j = CW * qq + u;
            const int buf = u & 1;
            if (q == qq) {
                double v = r[u];
                double d = rdlane(v, j);
                if (!(d > 0.0)) {
                    if (i == 0 && o + j < N) atomicCAS(status, 0, -(int)(o + j + 1));
                    d = 1.0;
                }
                const double ljj = sqrt(d);
                v = i > j ? v / ljj : (i == j ? ljj : 0.0);
                r[u] = v;
                col[buf][i] = v;
            }
            __syncthreads();
            // all CW broadcasts in flight together, then a branch-free update
            // (a predicated read per column would wait on each one in turn)
            const double lij = col[buf][i];
            double cv[CW];
#pragma unroll
            for (int uu = 0; uu < CW; ++uu) cv[uu] = col[buf][CW * q + uu];
#pragma unroll
            for (int uu = 0; uu < CW; ++uu) r[uu] = (CW * q + uu > j) ? r[uu] - lij * cv[uu] : r[uu];
        }
    }
#pragma unroll
    for (int u = 0; u < CW; ++u) {
        const int j = CW * q + u;
        A[(o + i) + (o + j) * Np] = i >= j ? r[u] : 0.0;
    }
}

// panel: A_ik <- A_ik L_kk^{-T} for the row blocks ib > kb, one wavefront per
// row block (lane = row, the row in registers), column by column:
//   x_c = a_c / L_cc,  then a_j -= x_c L_jc for j > c,
// with L_jc read as LDS broadcasts; a column's FMAs are independent of each
// other.  nz[ib] = the block is not all zero.
__global__ __launch_bounds__(GNT) void k_trsm_panel(double* __restrict__ A, int64_t Np, int kb, int nblk,
                                                    int* __restrict__ nz) {
    __shared__ double L[TB * TB];   // L_kk column-major: L[j + c * TB] = L_kk[j][c]
    const int64_t o = (int64_t)kb * TB;
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int j = e % TB, c = e / TB;
        L[e] = A[(o + j) + (o + c) * Np];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int ib = kb + 1 + (int)blockIdx.x * (GNT / 64) + (threadIdx.x >> 6);
    if (ib >= nblk) return;
    const int64_t r = (int64_t)ib * TB + lane;
    double x[TB];
#pragma unroll
    for (int c = 0; c < TB; ++c) x[c] = A[r + (o + c) * Np];
#pragma unroll
    for (int c = 0; c < TB; ++c) {
        __builtin_amdgcn_sched_barrier(0);   // one column's reads in flight at a time
        x[c] /= L[c + c * TB];
#pragma unroll
        for (int j = c + 1; j < TB; ++j) x[j] -= x[c] * L[j + c * TB];
    }
    int mine = 0;
#pragma unroll
    for (int c = 0; c < TB; ++c) {
        A[r + (o + c) * Np] = x[c];
        mine |= (x[c] != 0.0);
    }
    const int any = __any(mine);
    if (lane == 0) nz[ib] = any ? 1 : 0;
}

// trailing update A_ij -= L_ik L_jk^T over the lower tiles kb < jb <= ib on
// FP64 MFMA (16x16x4), skipped when either panel tile is exactly zero.  A
// wavefront computes a 32 x 32 quarter of the 64 x 64 tile as transposed
// blocks,  D[a][b] = sum_k L[rj + a][k] L[ri + b][k] = C[ri + b][rj + a],
// so that accumulator element v of lane l is C[ri + l%16][rj + l/16 + 4v]:
// the operand loads and the C reads and writes are all 16 consecutive
// doubles of a column.  Operands come straight from global memory (the
// panel stays in L2); the subtraction is folded in by negating the A operand.
// The tiles updated are those of the column blocks jb >= jlo (> kb), as many
// as the grid holds, column by column: one launch can take the next column
// block alone and another the rest.
__global__ __launch_bounds__(GNT) void k_syrk(double* __restrict__ A, int64_t Np, int kb, int jlo,
                                              int nblk, const int* __restrict__ nz) {
    // map blockIdx.x to (ib, jb) with jlo <= jb <= ib < nblk
    const int m = nblk - jlo;
    int idx = blockIdx.x, jj = 0;
    while (idx >= m - jj) {
        idx -= m - jj;
        ++jj;
    }
    const int jb = jlo + jj, ib = jb + idx;
    if (!nz[ib] || !nz[jb]) return;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int qi = wv & 1, qj = wv >> 1;
    if (ib == jb && qi < qj) return;   // the quarter above a diagonal tile's diagonal
    const int li = l & 15, lk = l >> 4;
    const int64_t o = (int64_t)kb * TB;
    const int64_t ri = (int64_t)ib * TB + 32 * qi, rj = (int64_t)jb * TB + 32 * qj;
    d4 acc[2][2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[bj][bi][v] = A[(ri + 16 * bi + li) + (rj + 16 * bj + lk + 4 * v) * Np];
    const double* __restrict__ pa = A + (rj + li) + (o + lk) * Np;
    const double* __restrict__ pb = A + (ri + li) + (o + lk) * Np;
#pragma unroll 4
    for (int k0 = 0; k0 < TB; k0 += 4) {
        const int64_t off = (int64_t)k0 * Np;
        const double a0 = -pa[off], a1 = -pa[off + 16];
        const double b0 = pb[off], b1 = pb[off + 16];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = ri + 16 * bi + li, gj = rj + 16 * bj + lk + 4 * v;
                if (ib != jb || gi >= gj) A[gi + gj * Np] = acc[bj][bi][v];
            }
}

// triangular solve with one TB x TB diagonal block for p columns:
//   lower (trans = 0):  L_kk X = B_k;   upper (trans = 1): L_kk^T X = B_k
// one wavefront per column, lane = row: once x_i is known (a broadcast from
// lane i) the lanes still to be solved subtract its contribution.
__global__ __launch_bounds__(GNT) void k_trsv_diag(const double* __restrict__ A, int64_t Np, int kb,
                                                   int trans, double* __restrict__ Bm, int p) {
    constexpr int LDL = TB + 1;
    __shared__ double L[TB * LDL];   // L[i + j * LDL] = L_kk[i][j]
    const int64_t o = (int64_t)kb * TB;
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int i = e % TB, j = e / TB;
        L[i + j * LDL] = A[(o + i) + (o + j) * Np];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int c = (int)blockIdx.x * (GNT / 64) + (threadIdx.x >> 6);
    if (c >= p) return;
    double* b = Bm + (int64_t)c * Np + o;
    double x = b[lane];
    // fully unrolled so that the LDS reads, which do not depend on x, are
    // issued ahead of the division chain
    if (!trans) {
#pragma unroll
        for (int i = 0; i < TB; ++i) {
            const double xi = rdlane(x, i) / L[i + i * LDL];
            if (lane == i) x = xi;
            else if (lane > i) x -= L[lane + i * LDL] * xi;
        }
    } else {
#pragma unroll
        for (int i = TB - 1; i >= 0; --i) {
            const double xi = rdlane(x, i) / L[i + i * LDL];
            if (lane == i) x = xi;
            else if (lane < i) x -= L[i + lane * LDL] * xi;
        }
    }
    b[lane] = x;
}

// block update after a diagonal solve at kb, for every other row block ib:
//   lower:  B_ib -= L_{ib,kb} X_kb  (ib > kb)
//   upper:  B_ib -= L_{kb,ib}^T X_kb (ib < kb)
__global__ __launch_bounds__(GNT) void k_trsv_update(const double* __restrict__ A, int64_t Np, int kb,
                                                     int trans, double* __restrict__ Bm, int p) {
    __shared__ double Lt[TB][TB + 1];
    __shared__ double Xs[MAXP][TB + 1];
    const int ib = trans ? (int)blockIdx.x : kb + 1 + (int)blockIdx.x;
    const int64_t o = (int64_t)kb * TB, r = (int64_t)ib * TB;
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int i = e % TB, j = e / TB;
        // Lt[i][j] = coefficient of X_kb[j] in row i of block ib
        Lt[i][j] = trans ? A[(o + j) + (r + i) * Np] : A[(r + i) + (o + j) * Np];
    }
    for (int e = threadIdx.x; e < p * TB; e += GNT) {
        const int c = e / TB, j = e % TB;
        Xs[c][j] = Bm[(int64_t)c * Np + o + j];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < p * TB; e += GNT) {
        const int c = e / TB, i = e % TB;
        double s = 0.0;
        for (int j = 0; j < TB; ++j) s += Lt[i][j] * Xs[c][j];
        Bm[(int64_t)c * Np + r + i] -= s;
    }
}

// Y = R(A0) X for a dense Np x Np matrix and p columns
__global__ __launch_bounds__(GNT) void k_gemm_rect(const double* __restrict__ A, int64_t Np,
                                                   const double* __restrict__ X, int p,
                                                   double* __restrict__ Y) {
    __shared__ double At[TB][TB + 1];
    __shared__ double Xs[MAXP][TB + 1];
    const int64_t r = (int64_t)blockIdx.x * TB;
    constexpr int PER = TB * MAXP / GNT;
    double acc[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) acc[e] = 0.0;
    for (int64_t c0 = 0; c0 < Np; c0 += TB) {
        for (int e = threadIdx.x; e < TB * TB; e += GNT) {
            const int i = e % TB, j = e / TB;
            At[i][j] = A[(r + i) + (c0 + j) * Np];
        }
        for (int e = threadIdx.x; e < p * TB; e += GNT) {
            const int c = e / TB, j = e % TB;
            Xs[c][j] = X[(int64_t)c * Np + c0 + j];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + e * GNT;
            const int i = idx % TB, c = idx / TB;
            if (c < p) {
                double s = 0.0;
                for (int j = 0; j < TB; ++j) s += At[i][j] * Xs[c][j];
                acc[e] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = threadIdx.x + e * GNT;
        const int i = idx % TB, c = idx / TB;
        if (c < p) Y[(int64_t)c * Np + r + i] = acc[e];
    }
}

// ------------------------------------------------------------ finalise
// per-workgroup partial sums of s1 = sum w and s2 = sum (tbar - t_n) w / span
__global__ __launch_bounds__(GNT) void k_sign_sums(const double* __restrict__ Y, int64_t Np, int64_t N,
                                                   int K, const double* __restrict__ t,
                                                   double* __restrict__ part) {
    __shared__ double red[GNT / 64][2 * MAXP];
    const int64_t n = (int64_t)blockIdx.x * GNT + threadIdx.x;
    const double tbar = 0.5 * (t[0] + t[N - 1]);
    const double span = N > 1 ? (t[N - 1] - t[0]) : 1.0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < K; ++k) {
        double a = 0.0, b = 0.0;
        if (n < N) {
            const double v = Y[(int64_t)k * Np + n];
            a = v;
            b = (tbar - t[n]) * v / span;
        }
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o, 64);
            b += __shfl_xor(b, o, 64);
        }
        if (lane == 0) {
            red[wv][2 * k] = a;
            red[wv][2 * k + 1] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * K) {
        double s = 0.0;
        for (int w = 0; w < GNT / 64; ++w) s += red[w][threadIdx.x];
        part[(int64_t)blockIdx.x * 2 * K + threadIdx.x] = s;
    }
}

// w[k*N + n] = sign_k * scale * Y[k][n];  lambda[k] = theta[k]
__global__ __launch_bounds__(GNT) void k_finalize(const double* __restrict__ Y, int64_t Np, int64_t N,
                                                  int K, double scale,
                                                  const double* __restrict__ part, int nwg,
                                                  const double* __restrict__ theta,
                                                  double* __restrict__ w,
                                                  double* __restrict__ lambda) {
    __shared__ double sg[MAXP];
    if (threadIdx.x < K) {
        double s1 = 0.0, s2 = 0.0;
        for (int g = 0; g < nwg; ++g) {
            s1 += part[(int64_t)g * 2 * K + 2 * threadIdx.x];
            s2 += part[(int64_t)g * 2 * K + 2 * threadIdx.x + 1];
        }
        const double key = fabs(s1) >= fabs(s2) ? s1 : s2;
        sg[threadIdx.x] = key < 0.0 ? -scale : scale;
        if (blockIdx.x == 0) lambda[threadIdx.x] = theta[threadIdx.x];
    }
    __syncthreads();
    const int64_t n = (int64_t)blockIdx.x * GNT + threadIdx.x;
    if (n >= N) return;
    for (int k = 0; k < K; ++k) w[(int64_t)k * N + n] = sg[k] * Y[(int64_t)k * Np + n];
}

// ------------------------------------------------------------ one sub-band
// The nominal band |f - fc0| <= f_w of a sub-band has the complex Hermitian
// R(A0) = e^{j 2 pi fc0 tau} sin(2 pi f_w tau) / (pi tau) (Sec. 3.2).  With D =
// diag(e^{j 2 pi fc0 (t_n - tc)}) and the real basis F0 of the band centred at
// 0 (k_lr_basis), R(A0) = (D F0)(D F0)^* to quadrature accuracy.  Columns
// j < Qn of F hold Re(D) F0_j, columns Qn + j hold Im(D) F0_j.
__global__ __launch_bounds__(256) void k_sb_basis(LrSeries d, double fc0) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= d.Np) return;
    const bool live = n < d.N;
    const double tn = live ? d.t[n] : d.tc;
    double cm = 0.0, sm = 0.0;
    if (live) {
        const double u = fc0 * (tn - d.tc);
        sincospi(2.0 * (u - rint(u)), &sm, &cm);
    }
    const int64_t im = (int64_t)d.Qn * d.Np;
    for (int q = 0; q < d.nq; ++q) {
        double c = 0.0, s = 0.0;
        if (live) {
            sincospi(2.0 * d.fw * d.glx[q] * (tn - d.tc), &s, &c);
            const double sq = sqrt(2.0 * d.fw * d.glx[MAXP + q]);
            c *= sq;
            s *= sq;
        }
        double* f = d.F + (int64_t)(2 * q) * d.Np + n;
        f[0] = cm * c;
        f[d.Np] = cm * s;
        f[im] = sm * c;
        f[im + d.Np] = sm * s;
    }
}

constexpr int HQ = MAXP / 2;   // largest complex rank of the sub-band path

__device__ __forceinline__ double wave_sum64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Eigen-decomposition of the complex Hermitian Gram G = X^* X (q x q, q even)
// of the sub-band path by Jacobi with the round-robin parallel ordering: each
// of the q - 1 steps of a sweep rotates q / 2 disjoint pairs at once (G <- G U,
// V <- V U by columns, then G <- U^* G by rows), four wavefronts sharing the
// updates.  P is the real Gram of [Xr Xi] (2q x 2q, row-major): G = (P_rr +
// P_ii) + j (P_ri - P_ir).  Rotation (p, r), p < r, with G_pr = m e^{j phi}:
// U = diag(1, e^{-j phi}) [[c, s], [-s, c]], t = s / c the smaller root of
// t^2 + 2 tau t - 1 = 0 with tau = (G_rr - G_pp) / (2 m), so that
// (U^* G U)_pr = 0.  A pair is rotated only when m > 1e-16 sqrt(G_pp G_rr);
// the sweeps stop after one without a rotation (60 at most).
// Out: theta [K] descending; Z (2q x 2K, column-major) for the real expansion
// [Xr Xi] Z: column k = [zr; -zi] / sqrt(theta_k) and column K + k =
// [zi; zr] / sqrt(theta_k) give the real and imaginary parts of
// X z_k / sqrt(theta_k).
constexpr int HJ_NT = 256;
__global__ __launch_bounds__(HJ_NT) void k_herm_jacobi(const double* __restrict__ P, int q, int K,
                                                       double* __restrict__ theta, double* __restrict__ Z) {
    __shared__ double Gr[HQ][HQ + 1], Gi[HQ][HQ + 1], Vr[HQ][HQ + 1], Vi[HQ][HQ + 1];
    __shared__ double rc[HQ / 2], rs[HQ / 2], rer[HQ / 2], rei[HQ / 2], rda[HQ / 2], rdd[HQ / 2];
    __shared__ int rp[HQ / 2], rr[HQ / 2], rot[HQ / 2];
    __shared__ int nrot;
    const int tid = threadIdx.x;
    const int p2 = 2 * q, h = q / 2, m = q - 1;
    for (int e = tid; e < q * q; e += HJ_NT) {
        const int a = e / q, b = e % q;
        Gr[a][b] = P[a * p2 + b] + P[(q + a) * p2 + q + b];
        Gi[a][b] = P[a * p2 + q + b] - P[(q + a) * p2 + b];
        Vr[a][b] = a == b ? 1.0 : 0.0;
        Vi[a][b] = 0.0;
    }
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        for (int st = 0; st < m; ++st) {
            if (tid < h) {
                const int k = tid;
                int p = k == 0 ? 0 : 1 + (st + k) % m;
                int r = 1 + (st - k + m) % m;
                if (p > r) {
                    const int x = p;
                    p = r;
                    r = x;
                }
                const double a = Gr[p][p], dd = Gr[r][r], br = Gr[p][r], bi = Gi[p][r];
                const double mm = sqrt(br * br + bi * bi);
                double c = 1.0, sn = 0.0, cph = 1.0, sph = 0.0, tt = 0.0;
                const bool doit = mm > 1e-16 * sqrt(fabs(a * dd)) && mm > 1e-300;
                if (doit) {
                    cph = br / mm;
                    sph = bi / mm;
                    const double tau = (dd - a) / (2.0 * mm);
                    tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    sn = tt * c;
                    atomicAdd(&nrot, 1);
                }
                rp[k] = p;
                rr[k] = r;
                rc[k] = c;
                rs[k] = sn;
                rer[k] = cph;
                rei[k] = sph;
                rda[k] = a - tt * mm;
                rdd[k] = dd + tt * mm;
                rot[k] = doit;
            }
            __syncthreads();
            // columns p, r of G and V: x U  (e^{-j phi} applied to column r)
            for (int e = tid; e < h * q; e += HJ_NT) {
                const int k = e / q, i = e % q;
                if (!rot[k]) continue;
                const int p = rp[k], r = rr[k];
                const double c = rc[k], sn = rs[k], cph = rer[k], sph = rei[k];
                double gr = Gr[i][r], gi = Gi[i][r];
                double er = cph * gr + sph * gi, ei = cph * gi - sph * gr;
                double gpr = Gr[i][p], gpi = Gi[i][p];
                Gr[i][p] = c * gpr - sn * er;
                Gi[i][p] = c * gpi - sn * ei;
                Gr[i][r] = sn * gpr + c * er;
                Gi[i][r] = sn * gpi + c * ei;
                gr = Vr[i][r];
                gi = Vi[i][r];
                er = cph * gr + sph * gi;
                ei = cph * gi - sph * gr;
                gpr = Vr[i][p];
                gpi = Vi[i][p];
                Vr[i][p] = c * gpr - sn * er;
                Vi[i][p] = c * gpi - sn * ei;
                Vr[i][r] = sn * gpr + c * er;
                Vi[i][r] = sn * gpi + c * ei;
            }
            __syncthreads();
            // rows p, r of G: U^* x  (e^{j phi} applied to row r)
            for (int e = tid; e < h * q; e += HJ_NT) {
                const int k = e / q, j = e % q;
                if (!rot[k]) continue;
                const int p = rp[k], r = rr[k];
                const double c = rc[k], sn = rs[k], cph = rer[k], sph = rei[k];
                const double hr = Gr[r][j], hi = Gi[r][j];
                const double fr = cph * hr - sph * hi, fi = cph * hi + sph * hr;
                const double gpr = Gr[p][j], gpi = Gi[p][j];
                Gr[p][j] = c * gpr - sn * fr;
                Gi[p][j] = c * gpi - sn * fi;
                Gr[r][j] = sn * gpr + c * fr;
                Gi[r][j] = sn * gpi + c * fi;
            }
            __syncthreads();
            if (tid < h && rot[tid]) {
                const int p = rp[tid], r = rr[tid];
                Gr[p][p] = rda[tid];
                Gr[r][r] = rdd[tid];
                Gi[p][p] = 0.0;
                Gi[r][r] = 0.0;
                Gr[p][r] = 0.0;
                Gi[p][r] = 0.0;
                Gr[r][p] = 0.0;
                Gi[r][p] = 0.0;
            }
            __syncthreads();
        }
        const int nr = nrot;
        __syncthreads();
        if (tid == 0) nrot = 0;
        __syncthreads();
        if (nr == 0) break;
    }
    if (tid >= 64) return;
    // the K largest, ties to the lower index (wavefront 0)
    const int l = tid;
    double ev = l < q ? Gr[l][l] : -DBL_MAX;
    for (int k = 0; k < K; ++k) {
        double bv = ev;
        int bx = l;
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, 64);
            const int ox = __shfl_xor(bx, o, 64);
            if (ov > bv || (ov == bv && ox < bx)) {
                bv = ov;
                bx = ox;
            }
        }
        if (l == 0) theta[k] = bv;
        if (l < q) {
            const double sc = bv > 0.0 ? 1.0 / sqrt(bv) : 0.0;
            const double zr = Vr[l][bx] * sc, zi = Vi[l][bx] * sc;
            Z[l + (int64_t)k * p2] = zr;
            Z[q + l + (int64_t)k * p2] = -zi;
            Z[l + (int64_t)(K + k) * p2] = zi;
            Z[q + l + (int64_t)(K + k) * p2] = zr;
        }
        if (l == bx) ev = -DBL_MAX;
    }
}

// per-workgroup partial sums for the phase of complex taper k (real part in
// row k of Y, imaginary part in row K + k): with v_n = y_n e^{-j 2 pi fc0
// (t_n - tbar)}, a = sum v_n and b = sum (tbar - t_n) v_n / span
__global__ __launch_bounds__(GNT) void k_phase_sums(const double* __restrict__ Y, int64_t Np, int64_t N,
                                                    int K, const double* __restrict__ t, double fc0,
                                                    double* __restrict__ part) {
    __shared__ double red[GNT / 64][4 * HQ];
    const int64_t n = (int64_t)blockIdx.x * GNT + threadIdx.x;
    const double tbar = 0.5 * (t[0] + t[N - 1]);
    const double span = N > 1 ? (t[N - 1] - t[0]) : 1.0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double cm = 1.0, sm = 0.0, lev = 0.0;
    if (n < N) {
        const double u = fc0 * (t[n] - tbar);
        sincospi(2.0 * (u - rint(u)), &sm, &cm);
        lev = (tbar - t[n]) / span;
    }
    for (int k = 0; k < K; ++k) {
        double ar = 0.0, ai = 0.0;
        if (n < N) {
            const double wr = Y[(int64_t)k * Np + n], wi = Y[(int64_t)(K + k) * Np + n];
            ar = wr * cm + wi * sm;
            ai = wi * cm - wr * sm;
        }
        double br = lev * ar, bi = lev * ai;
        ar = wave_sum64(ar);
        ai = wave_sum64(ai);
        br = wave_sum64(br);
        bi = wave_sum64(bi);
        if (lane == 0) {
            red[wv][4 * k] = ar;
            red[wv][4 * k + 1] = ai;
            red[wv][4 * k + 2] = br;
            red[wv][4 * k + 3] = bi;
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 * K) {
        double s = 0.0;
        for (int w = 0; w < GNT / 64; ++w) s += red[w][threadIdx.x];
        part[(int64_t)blockIdx.x * 4 * K + threadIdx.x] = s;
    }
}

// planar complex tapers: w[k N + n] = Re, w[(K + k) N + n] = Im of
// scale * y_k * conj(key_k) / |key_k|, key_k the one of a_k, b_k with the
// larger modulus (a_k on ties); lambda[k] = theta[k]
__global__ __launch_bounds__(GNT) void k_finalize_c(const double* __restrict__ Y, int64_t Np, int64_t N,
                                                    int K, double scale, const double* __restrict__ part,
                                                    int nwg, const double* __restrict__ theta,
                                                    double* __restrict__ w, double* __restrict__ lambda) {
    __shared__ double phr[HQ], phi[HQ];
    if (threadIdx.x < K) {
        const int k = threadIdx.x;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int g = 0; g < nwg; ++g)
            for (int c = 0; c < 4; ++c) a[c] += part[(int64_t)g * 4 * K + 4 * k + c];
        const double ma = sqrt(a[0] * a[0] + a[1] * a[1]), mb = sqrt(a[2] * a[2] + a[3] * a[3]);
        const bool useb = !(ma >= mb);
        const double kr = useb ? a[2] : a[0], ki = useb ? a[3] : a[1], mk = useb ? mb : ma;
        phr[k] = mk > 0.0 ? scale * kr / mk : scale;
        phi[k] = mk > 0.0 ? -scale * ki / mk : 0.0;
        if (blockIdx.x == 0) lambda[k] = theta[k];
    }
    __syncthreads();
    const int64_t n = (int64_t)blockIdx.x * GNT + threadIdx.x;
    if (n >= N) return;
    for (int k = 0; k < K; ++k) {
        const double yr = Y[(int64_t)k * Np + n], yi = Y[(int64_t)(K + k) * Np + n];
        w[(int64_t)k * N + n] = phr[k] * yr - phi[k] * yi;
        w[(int64_t)(K + k) * N + n] = phr[k] * yi + phi[k] * yr;
    }
}

// ------------------------------------------------------------ host side

int ilog2i(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

std::vector<cplx<double>> twiddles64(int64_t n, int64_t count, int64_t stride) {
    std::vector<cplx<double>> v(count);
    for (int64_t j = 0; j < count; ++j) {
        const long double a = -2.0L * (long double)M_PI * (long double)((j * stride) % n) / (long double)n;
        v[j] = {(double)cosl(a), (double)sinl(a)};
    }
    return v;
}

int upload64(Ctx* ctx, DevBuf& b, const std::vector<cplx<double>>& v) {
    M2N_TRY(ctx->alloc(b, v.size() * sizeof(cplx<double>)));
    M2N_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(cplx<double>), hipMemcpyHostToDevice));
    return M2N_OK;
}

void release_fft(Ctx* ctx, FftPlan64& f) {
    ctx->release(f.tw);
    ctx->release(f.tw_lo);
    ctx->release(f.tw_hi);
}

int make_fft64(Ctx* ctx, int64_t M, FftPlan64& f) {
    f.M = M;
    f.log_M = ilog2i(M);
    f.single = M <= 4096;
    if (f.single) {
        f.tw_len = (int)M;
        return upload64(ctx, f.tw, twiddles64(M, M, 1));
    }
    int l1 = f.log_M / 2;
    if (l1 > 10) l1 = 10;
    f.N1 = 1 << l1;
    f.N2 = (int)(M / f.N1);
    if (f.N2 > 4096) {
        set_error("lattice span too long for this build (M = %lld)", (long long)M);
        return M2N_ERR_UNSUPPORTED;
    }
    f.BB = 65536 / (f.N1 * 16);
    if (f.BB > 16) f.BB = 16;
    f.MM = 65536 / (f.N2 * 16);
    if (f.MM > 16) f.MM = 16;
    f.lo_bits = (f.log_M + 1) / 2;
    f.tw_len = f.N1 > f.N2 ? f.N1 : f.N2;
    M2N_TRY(upload64(ctx, f.tw, twiddles64(f.tw_len, f.tw_len, 1)));
    M2N_TRY(upload64(ctx, f.tw_lo, twiddles64(M, int64_t(1) << f.lo_bits, 1)));
    M2N_TRY(upload64(ctx, f.tw_hi, twiddles64(M, M >> f.lo_bits, int64_t(1) << f.lo_bits)));
    return M2N_OK;
}

// run the FFT of `batch` sequences of length M from (smode) to (dmode)
int run_fft64(const FftPlan64& f, hipStream_t st, const ConvArgs& a, int batch, int smode, int dmode,
              cplx<double>* inter) {
    if (f.single) {
#define M2N_FS(MV)                                                                        \
    case MV:                                                                              \
        hipLaunchKernelGGL((k_fft_small<MV>), dim3(batch), dim3(GNT), 0, st, a, smode,     \
                           dmode, (const cplx<double>*)f.tw.p);                           \
        break;
        switch (f.M) {
            M2N_FS(64) M2N_FS(128) M2N_FS(256) M2N_FS(512) M2N_FS(1024) M2N_FS(2048) M2N_FS(4096)
            default:
                set_error("bad small FFT size %lld", (long long)f.M);
                return M2N_ERR_UNSUPPORTED;
        }
#undef M2N_FS
        M2N_HIP(hipGetLastError());
        return M2N_OK;
    }
    const int log_N2 = ilog2i(f.N2);
    bool done = false;
#define M2N_FA(N1V, BV)                                                                         \
    if (!done && f.N1 == N1V && f.BB == BV) {                                                   \
        hipLaunchKernelGGL((k_fftA<N1V, BV>), dim3((unsigned)(batch * (f.N2 / BV))), dim3(GNT), \
                           0, st, a, smode, log_N2, f.M, (const cplx<double>*)f.tw.p,            \
                           f.tw_len / N1V, (const cplx<double>*)f.tw_lo.p,                      \
                           (const cplx<double>*)f.tw_hi.p, f.lo_bits, inter);                   \
        done = true;                                                                            \
    }
    M2N_FA(64, 16) M2N_FA(128, 16) M2N_FA(256, 16) M2N_FA(512, 8) M2N_FA(1024, 4)
#undef M2N_FA
    if (!done) {
        set_error("no FFT pass-A kernel for N1 = %d", f.N1);
        return M2N_ERR_UNSUPPORTED;
    }
    M2N_HIP(hipGetLastError());
    done = false;
#define M2N_FB(N2V, MV)                                                                        \
    if (!done && f.N2 == N2V && f.MM == MV) {                                                  \
        hipLaunchKernelGGL((k_fftB<N2V, MV>), dim3((unsigned)(batch * (f.N1 / MV))), dim3(GNT), \
                           0, st, a, dmode, f.N1, f.M, (const cplx<double>*)inter,             \
                           (const cplx<double>*)f.tw.p, f.tw_len / N2V);                      \
        done = true;                                                                           \
    }
    M2N_FB(64, 16) M2N_FB(128, 16) M2N_FB(256, 16) M2N_FB(512, 8) M2N_FB(1024, 4)
    M2N_FB(2048, 2) M2N_FB(4096, 1)
#undef M2N_FB
    if (!done) {
        set_error("no FFT pass-B kernel for N2 = %d", f.N2);
        return M2N_ERR_UNSUPPORTED;
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

struct Solver {
    Ctx* ctx;
    hipStream_t st;
    int64_t N, Np;
    int p, K;
    // lattice
    bool lattice = false;
    const FftPlan64* fft = nullptr;
    int* map = nullptr;
    double* Hhat = nullptr;
    cplx<double>* cbuf1 = nullptr;   // pass-A output / natural-order temp
    cplx<double>* cbuf2 = nullptr;
    // dense
    double* RB = nullptr;
    double* RA = nullptr;
    double* tmp = nullptr;
    int* nz = nullptr;
    int nblk = 0;

    int apply(const double* V, double* W) {
        if (lattice) {
            const int pairs = (p + 1) / 2;
            ConvArgs a{};
            a.V = V;
            a.map = map;
            a.Np = Np;
            a.p = p;
            a.Hhat = Hhat;
            a.Y = W;
            M2N_PROF(ctx, st, "toeplitz_fft_conv");
            if (fft->single) {
                // whole convolution in two single-workgroup transforms
                a.dst = cbuf1;
                M2N_TRY(run_fft64(*fft, st, a, pairs, SRC_PAIR, DST_MULCONJ, nullptr));
                a.src = cbuf1;
                M2N_TRY(run_fft64(*fft, st, a, pairs, SRC_DIRECT, DST_PAIR, nullptr));
            } else {
                a.dst = cbuf1;
                M2N_TRY(run_fft64(*fft, st, a, pairs, SRC_PAIR, DST_MULCONJ, cbuf2));
                a.src = cbuf1;
                M2N_TRY(run_fft64(*fft, st, a, pairs, SRC_DIRECT, DST_PAIR, cbuf2));
            }
            return M2N_OK;
        }
        // dense: tmp = L^{-T} V; W = R(A0) tmp; W = L^{-1} W
        M2N_HIP(hipMemcpyAsync(tmp, V, sizeof(double) * (size_t)p * Np, hipMemcpyDeviceToDevice, st));
        M2N_TRY(trsv(tmp, 1));
        {
            M2N_PROF(ctx, st, "k_gemm_rect");
            hipLaunchKernelGGL(k_gemm_rect, dim3((unsigned)nblk), dim3(GNT), 0, st, RA, Np, tmp, p, W);
        }
        M2N_HIP(hipGetLastError());
        M2N_TRY(trsv(W, 0));
        return M2N_OK;
    }

    // in-place block triangular solve with L (trans = 0) or L^T (trans = 1)
    int trsv(double* Bm, int trans) {
        for (int s = 0; s < nblk; ++s) {
            const int kb = trans ? nblk - 1 - s : s;
            {
                M2N_PROF(ctx, st, "k_trsv_diag");
                hipLaunchKernelGGL(k_trsv_diag, dim3((unsigned)((p + 3) / 4)), dim3(GNT), 0, st, RB, Np, kb,
                                   trans, Bm, p);
            }
            const int nupd = trans ? kb : nblk - kb - 1;
            if (nupd > 0)
                {
                    M2N_PROF(ctx, st, "k_trsv_update");
                    hipLaunchKernelGGL(k_trsv_update, dim3((unsigned)nupd), dim3(GNT), 0, st, RB, Np, kb,
                                       trans, Bm, p);
                }
        }
        M2N_HIP(hipGetLastError());
        return M2N_OK;
    }
};

// block subspace iteration with Rayleigh-Ritz; returns the Ritz vectors of
// the K largest eigenvalues in Y (orthonormal) and theta.
int subspace_solve(Solver& S, double* V, double* W, double* Y, double* gacc, double* res,
                   double* Q, double* th, int64_t nchunks) {
    Ctx* ctx = S.ctx;
    hipStream_t st = S.st;
    const int64_t N = S.N, Np = S.Np;
    const int p = S.p, K = S.K;
    const int gram_wg = (int)(nchunks < GRAM_WG_MAX ? nchunks : GRAM_WG_MAX);
    const int cpw = (int)((nchunks + gram_wg - 1) / gram_wg);
    const int row_wg = (int)((Np + 63) / 64);
    const int pc = (p + 7) / 8 * 8;
    void* vpart;
    M2N_TRY(ctx->workspace("gep_gpart", sizeof(double) * (size_t)gram_wg * 2 * p * p, &vpart));
    {
        M2N_PROF(ctx, st, "k_randinit");
        dim3 g2((unsigned)((Np + 255) / 256), (unsigned)p);
        hipLaunchKernelGGL(k_randinit, g2, dim3(256), 0, st, V, Np, N, p, (uint64_t)0x5EED);
    }
    M2N_HIP(hipGetLastError());
    std::vector<double> hres((size_t)row_wg * K);
    double prev = 1e300;
    for (int it = 0; it < 40; ++it) {
        M2N_TRY(S.apply(V, W));
        {
            M2N_PROF(ctx, st, "k_gram2");
            hipLaunchKernelGGL(k_gram2, dim3(gram_wg), dim3(GNT), 0, st, V, W, Np, N, p, cpw, nchunks,
                               2, (double*)vpart);
            hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)((2 * p * p + 63) / 64)), dim3(256), 0,
                               st, (const double*)vpart, gram_wg, 2 * p * p, gacc);
        }
        {
            M2N_PROF(ctx, st, "k_small_rr");
            if (p <= 16) hipLaunchKernelGGL(k_small_rr<16>, dim3(1), dim3(64), 0, st, gacc, p, Q, th);
            else if (p <= 32) hipLaunchKernelGGL(k_small_rr<32>, dim3(1), dim3(64), 0, st, gacc, p, Q, th);
            else if (p <= 48) hipLaunchKernelGGL(k_small_rr<48>, dim3(1), dim3(64), 0, st, gacc, p, Q, th);
            else hipLaunchKernelGGL(k_small_rr<64>, dim3(1), dim3(64), 0, st, gacc, p, Q, th);
        }
        {
            M2N_PROF(ctx, st, "k_rotate2");
#define M2N_ROT(PCV)                                                                            \
    case PCV:                                                                                   \
        hipLaunchKernelGGL(k_rotate2<PCV>, dim3(row_wg), dim3(64), 0, st, V, W, Q, th, Np, N, p, \
                           K, Y, res);                                                          \
        break;
            switch (pc) {
                M2N_ROT(8) M2N_ROT(16) M2N_ROT(24) M2N_ROT(32) M2N_ROT(40) M2N_ROT(48) M2N_ROT(56)
                M2N_ROT(64)
                default:
                    set_error("internal: block width %d", p);
                    return M2N_ERR_ARG;
            }
#undef M2N_ROT
        }
        M2N_HIP(hipGetLastError());
        if (it == 0 && p < N) continue;   // a random start is never converged
        M2N_HIP(hipMemcpyAsync(hres.data(), res, sizeof(double) * hres.size(), hipMemcpyDeviceToHost,
                               st));
        M2N_HIP(hipStreamSynchronize(st));
        double rmax = 0.0;
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int g = 0; g < row_wg; ++g) s += hres[(size_t)g * K + k];
            rmax = std::fmax(rmax, std::sqrt(s));
        }
        if (!std::isfinite(rmax)) break;
        if (p == N || rmax <= 1e-13 || (it >= 3 && rmax > 0.5 * prev && rmax <= 1e-10))
            return M2N_OK;
        prev = rmax;
    }
    set_error("subspace iteration did not converge");
    return M2N_ERR_NO_CONVERGE;
}

}  // namespace

// Gram partials on the matrix cores and their fixed-order reduction
int launch_gram_mfma(Ctx* ctx, hipStream_t st, int maxpF, int maxred, int ns, const LrSeries& d0,
                     const LrSeries* D) {
    {
        M2N_PROF(ctx, st, "k_gram_mfma");
        const int nt = (maxpF + 15) / 16;
        const dim3 g((unsigned)maxred, (unsigned)ns);
        if (nt == 1) hipLaunchKernelGGL(k_gram_mfma<1>, g, dim3(64), 0, st, d0, D);
        else if (nt == 2) hipLaunchKernelGGL(k_gram_mfma<2>, g, dim3(64), 0, st, d0, D);
        else if (nt == 3) hipLaunchKernelGGL(k_gram_mfma<3>, g, dim3(64), 0, st, d0, D);
        else hipLaunchKernelGGL(k_gram_mfma<4>, g, dim3(64), 0, st, d0, D);
    }
    {
        M2N_PROF(ctx, st, "k_gram_reduce");
        hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((maxpF * maxpF + 63) / 64), (unsigned)ns),
                           dim3(512), 0, st, d0, D);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

int launch_lr_expand(Ctx* ctx, hipStream_t st, int maxq, int64_t blocks, int ns, const LrSeries& d0,
                     const LrSeries* D) {
    M2N_PROF(ctx, st, "k_lr_expand");
    const dim3 g((unsigned)blocks, (unsigned)ns);
    switch ((maxq + 7) / 8 * 8) {
        case 8: hipLaunchKernelGGL(k_lr_expand<8>, g, dim3(64), 0, st, d0, D); break;
        case 16: hipLaunchKernelGGL(k_lr_expand<16>, g, dim3(64), 0, st, d0, D); break;
        case 24: hipLaunchKernelGGL(k_lr_expand<24>, g, dim3(64), 0, st, d0, D); break;
        case 32: hipLaunchKernelGGL(k_lr_expand<32>, g, dim3(64), 0, st, d0, D); break;
        case 40: hipLaunchKernelGGL(k_lr_expand<40>, g, dim3(64), 0, st, d0, D); break;
        case 48: hipLaunchKernelGGL(k_lr_expand<48>, g, dim3(64), 0, st, d0, D); break;
        case 56: hipLaunchKernelGGL(k_lr_expand<56>, g, dim3(64), 0, st, d0, D); break;
        case 64: hipLaunchKernelGGL(k_lr_expand<64>, g, dim3(64), 0, st, d0, D); break;
        default:
            set_error("internal: quadrature rank %d", maxq);
            return M2N_ERR_ARG;
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

// Gauss-Legendre table (positive nodes, then weights at + MAXP) of order Q,
// uploaded once per context
int gl_table(Ctx* ctx, int Q, const double** out) {
    auto itg = ctx->gl.find(Q);
    if (itg == ctx->gl.end()) {
        std::vector<double> gx, gw, tab(2 * MAXP, 0.0);
        gauss_legendre(Q, gx, gw);
        int j = 0;
        for (int i = 0; i < Q; ++i)
            if (gx[i] > 0.0) {
                tab[j] = gx[i];
                tab[MAXP + j] = gw[i];
                ++j;
            }
        DevBuf b;
        M2N_TRY(ctx->alloc(b, sizeof(double) * 2 * MAXP));
        M2N_HIP(hipMemcpy(b.p, tab.data(), sizeof(double) * 2 * MAXP, hipMemcpyHostToDevice));
        itg = ctx->gl.emplace(Q, b).first;
    }
    *out = (const double*)itg->second.p;
    return M2N_OK;
}

// quadrature rank of R(A0): Gauss-Legendre in f over [-fw, fw]; the
// integrand e^{j 2 pi f tau} turns through at most beta = 2 pi fw span
// radians, and 0.7 beta + 14 nodes reach rounding level for beta <= 90
int quad_rank(double fw, double span, int K) {
    const double beta = 2.0 * M_PI * fw * span;
    int Qn = (int)std::ceil(0.7 * beta) + 14;
    if (Qn < K + 2) Qn = K + 2;
    return Qn + (Qn & 1);
}

// what the t check found for one series
struct TStat {
    int flags = 0;
    unsigned long long first_nonfinite = ~0ull, first_order = ~0ull;
    double t0 = 0, tN = 0;
};

// Launch the check of the sampling times of every series (one launch); the
// records land in the pinned host record and are read by t_check_read once
// the stream has passed the launch.
int t_check_launch(Ctx* ctx, hipStream_t st, const GepIn* in, int ns, std::vector<TaSeries>& ds) {
    ds.assign(ns, TaSeries());
    size_t ninfo = 0;
    int maxblk = 1;
    for (int i = 0; i < ns; ++i) {
        const int64_t N = in[i].N;
        TaSeries& d = ds[i];
        d.t = in[i].t;
        d.N = N;
        d.per_wg = N <= 256 * 256 ? 256 : (N + 255) / 256;
        d.nblk = (int)((N + d.per_wg - 1) / d.per_wg);
        d.pad = 0;
        ninfo += (size_t)d.nblk;
        maxblk = std::max(maxblk, d.nblk);
    }
    const size_t hdr_bytes = ((size_t)ns * 2 * sizeof(double) + 255) & ~size_t(255);
    M2N_TRY(ctx->pinned_info(hdr_bytes + ninfo * sizeof(TInfo)));
    double* hdr = (double*)ctx->hinfo;
    TInfo* info = (TInfo*)((char*)ctx->hinfo + hdr_bytes);
    size_t o = 0;
    for (int i = 0; i < ns; ++i) {
        ds[i].hdr = hdr + 2 * i;
        ds[i].info = info + o;
        o += (size_t)ds[i].nblk;
    }
    const TaSeries* D = nullptr;
    if (ns > 1) {
        void* vd;
        M2N_TRY(ctx->workspace("gep_tdesc", sizeof(TaSeries) * (size_t)ns, &vd));
        M2N_TRY(ctx->stage(st, ds.data(), sizeof(TaSeries) * (size_t)ns, vd));
        D = (const TaSeries*)vd;
    }
    {
        M2N_PROF(ctx, st, "k_t_analyze");
        hipLaunchKernelGGL(k_t_analyze, dim3((unsigned)maxblk, (unsigned)ns), dim3(256), 0, st, ds[0], D);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

void t_check_read(const std::vector<TaSeries>& ds, std::vector<TStat>& out) {
    const int ns = (int)ds.size();
    out.assign(ns, TStat());
    for (int i = 0; i < ns; ++i) {
        TStat& r = out[i];
        for (int g = 0; g < ds[i].nblk; ++g) {
            const TInfo& f = ds[i].info[g];
            r.flags |= f.flags;
            r.first_nonfinite = std::min(r.first_nonfinite, f.first_nonfinite);
            r.first_order = std::min(r.first_order, f.first_order);
        }
        r.t0 = ds[i].hdr[0];
        r.tN = ds[i].hdr[1];
    }
}

// Check the sampling times of every series on the device (one launch) and
// wait for the records: one host round trip for the whole set.
int t_check(Ctx* ctx, hipStream_t st, const GepIn* in, int ns, std::vector<TStat>& out) {
    std::vector<TaSeries> ds;
    M2N_TRY(t_check_launch(ctx, st, in, ns, ds));
    M2N_HIP(hipStreamSynchronize(st));
    t_check_read(ds, out);
    return M2N_OK;
}

int t_status(const TStat& r, int series) {
    if (r.flags & 1) {
        set_error("series %d: non-finite sampling time at %llu", series, r.first_nonfinite);
        return M2N_ERR_ARG;
    }
    if (r.flags & 2) {
        set_error("series %d: sampling times not strictly increasing at %llu", series, r.first_order);
        return M2N_ERR_T_ORDER;
    }
    return M2N_OK;
}

bool on_lattice(const GepIn& s, const TStat& r) {
    const double cB = 2.0 * s.fmax;
    return !(r.flags & 4) && cB == std::rint(cB) && cB >= 1.0 && (r.tN - r.t0) < 2.0e6;
}

// R(B) = c I and Q + 2 <= 64: the batched low-rank path
bool lattice_lowrank(const GepIn& s, const TStat& r) {
    if (!on_lattice(s, r)) return false;
    const double span = s.N > 1 ? r.tN - r.t0 : 0.0;
    return quad_rank(s.fw, span, s.K) + 2 <= MAXP;
}

// The K largest generalized eigenpairs for series whose R(B) is c I, all in
// one set of launches: quadrature basis F = [cos | sin | 1 | tau], its Gram
// matrix on the matrix cores, the Q x Q eigenproblem with the sign and the
// scale folded in, and the expansion straight into the caller's tapers.
int gep_lattice_batch(Ctx* ctx, hipStream_t st, const GepIn* in, const TStat* stat,
                      const std::vector<int>& idx) {
    const int ns = (int)idx.size();
    if (ns == 0) return M2N_OK;
    std::vector<LrSeries> ds(ns);
    int maxq = 0, maxpF = 0, maxred = 0;
    int64_t maxNp = 0, maxN = 0;
    for (int j = 0; j < ns; ++j) {
        const GepIn& g = in[idx[j]];
        const TStat& r = stat[idx[j]];
        LrSeries& d = ds[j];
        std::memset(&d, 0, sizeof(d));
        const double cB = 2.0 * g.fmax;
        const double span = g.N > 1 ? r.tN - r.t0 : 0.0;
        d.t = g.t;
        d.N = g.N;
        d.Np = (g.N + TB - 1) / TB * TB;
        d.ldy = g.N;
        d.tc = 0.5 * (r.t0 + r.tN);
        d.span = span > 0.0 ? span : 1.0;
        d.fw = g.fw;
        d.scale = 1.0 / cB;
        d.wscale = std::sqrt(2.0 * g.fw) / cB;
        d.c = cB;
        d.K = g.K;
        d.Qn = quad_rank(g.fw, span, g.K);
        d.pF = d.Qn + 2;
        d.nq = d.Qn / 2;
        d.fuse = 1;
        d.nchunks = (int)((d.Np + GRAM_ROWS - 1) / GRAM_ROWS);
        d.theta = g.lambda;
        d.Y = g.w;
        M2N_TRY(gl_table(ctx, d.Qn, &d.glx));
        maxq = std::max(maxq, d.Qn);
        maxpF = std::max(maxpF, d.pF);
        maxNp = std::max(maxNp, d.Np);
        maxN = std::max(maxN, d.N);
    }
    // 64-row chunks per Gram wavefront: one for a single series (up to 512
    // wavefronts), more in a batch so that about 2048 wavefronts run and
    // few partial Gram matrices are written and summed
    int64_t chunks = 0;
    for (auto& d : ds) chunks += d.nchunks;
    const int cpw_b = (int)std::max<int64_t>(1, chunks / 2048);
    for (auto& d : ds) {
        d.cpw = std::max(cpw_b, (d.nchunks + 511) / 512);
        d.nred = (d.nchunks + d.cpw - 1) / d.cpw;
        maxred = std::max(maxred, d.nred);
    }
    // workspace: F, Gram partials, Gram, Z per series (256-byte aligned)
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t tot = 0;
    for (auto& d : ds)
        tot += al(sizeof(double) * (size_t)d.pF * d.Np) + al(sizeof(double) * (size_t)d.nred * d.pF * d.pF) +
               al(sizeof(double) * (size_t)d.pF * d.pF) + al(sizeof(double) * (size_t)d.Qn * d.K);
    void* vw;
    M2N_TRY(ctx->workspace("gep_lr", tot, &vw));
    char* cur = (char*)vw;
    for (auto& d : ds) {
        d.F = (double*)cur;
        cur += al(sizeof(double) * (size_t)d.pF * d.Np);
        d.gpart = (double*)cur;
        cur += al(sizeof(double) * (size_t)d.nred * d.pF * d.pF);
        d.G = (double*)cur;
        cur += al(sizeof(double) * (size_t)d.pF * d.pF);
        d.Z = (double*)cur;
        cur += al(sizeof(double) * (size_t)d.Qn * d.K);
    }
    const LrSeries* D = nullptr;
    if (ns > 1) {
        void* vd;
        M2N_TRY(ctx->workspace("gep_lrdesc", sizeof(LrSeries) * (size_t)ns, &vd));
        M2N_TRY(ctx->stage(st, ds.data(), sizeof(LrSeries) * (size_t)ns, vd));
        D = (const LrSeries*)vd;
    }
    const LrSeries& d0 = ds[0];
    const unsigned ys = (unsigned)ns;
    {
        M2N_PROF(ctx, st, "k_lr_basis");
        hipLaunchKernelGGL(k_lr_basis, dim3((unsigned)((maxNp + 255) / 256), (unsigned)((maxq / 2 + 1 + LR_QB - 1) / LR_QB), ys),
                           dim3(256), 0, st, d0, D);
    }
    M2N_HIP(hipGetLastError());
    M2N_TRY(launch_gram_mfma(ctx, st, maxpF, maxred, ns, d0, D));
    {
        M2N_PROF(ctx, st, "k_sym_topk");
        launch_sym_topk(st, maxq, ns, d0, D);
    }
    M2N_TRY(launch_lr_expand(ctx, st, maxq, (maxN + 63) / 64, ns, d0, D));
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

// One series by the dense (R(B) not c I) or wide-band (Q + 2 > 64) paths.
// R(B) = L L^T in S.RB by the tiled Cholesky (zero tiles skipped): the full
// band |f| <= f_max when fmin = 0, else the sub-band f_min <= |f| <= f_max.
// Blocks on the pivot status; M2N_ERR_NOT_PD when a pivot is <= 0.
int factor_dense(Ctx* ctx, hipStream_t st, Solver& S, const double* td, int64_t N, double fmin,
                 double fmax) {
    const int64_t Np = S.Np;
    if (Np > 65536) {
        set_error("dense GEP limited to N <= 65536 in this build");
        return M2N_ERR_UNSUPPORTED;
    }
    S.nblk = (int)(Np / TB);
    void *vRB, *vnz, *vst;
    M2N_TRY(ctx->workspace("gep_RB", sizeof(double) * (size_t)Np * Np, &vRB));
    M2N_TRY(ctx->workspace("gep_nz", sizeof(int) * (size_t)S.nblk * 2, &vnz));
    M2N_TRY(ctx->workspace("gep_status", 64, &vst));
    S.RB = (double*)vRB;
    S.nz = (int*)vnz;
    M2N_HIP(hipMemsetAsync(vst, 0, 64, st));
    {
        dim3 gs((unsigned)((Np + 255) / 256), (unsigned)Np);
        if (fmin == 0.0) {
            M2N_PROF(ctx, st, "k_gen_sinc");
            hipLaunchKernelGGL(k_gen_sinc, gs, dim3(256), 0, st, td, N, Np, fmax, 1.0, S.RB);
        } else {
            M2N_PROF(ctx, st, "k_gen_subband");
            hipLaunchKernelGGL(k_gen_subband, gs, dim3(256), 0, st, td, N, Np, fmin, fmax, S.RB);
        }
    }
    M2N_HIP(hipGetLastError());
    // Right-looking with a look-ahead of one panel: the update of column
    // block kb + 1 by panel kb runs first on st, then the rest of that
    // update on the second stream while st factors panel kb + 1 (the
    // panel kernels use a few compute units; the rest of the update
    // fills the others); st waits for it before panel kb + 1's update.
    // The zero-tile flags of panel kb are nz[(kb & 1) nblk + ib], so that
    // panel kb + 1's flags do not overwrite those still being read.
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    M2N_TRY(ctx->aux_stream(&s2, &ev_fork, &ev_join));
    auto potrf = [&](int kb) {
        M2N_PROF(ctx, st, "k_potrf");
        hipLaunchKernelGGL(k_potrf, dim3(1), dim3(4 * TB), 0, st, S.RB, Np, kb, N, (int*)vst);
    };
    auto trsm = [&](int kb) {
        const int rem = S.nblk - kb - 1;
        M2N_PROF(ctx, st, "k_trsm_panel");
        hipLaunchKernelGGL(k_trsm_panel, dim3((unsigned)((rem + 3) / 4)), dim3(GNT), 0, st, S.RB, Np,
                           kb, S.nblk, S.nz + (kb & 1) * S.nblk);
    };
    potrf(0);
    if (S.nblk > 1) trsm(0);
    for (int kb = 0; kb + 1 < S.nblk; ++kb) {
        const int rem = S.nblk - kb - 1;
        const int* nzk = S.nz + (kb & 1) * S.nblk;
        {
            M2N_PROF(ctx, st, "k_syrk");
            hipLaunchKernelGGL(k_syrk, dim3((unsigned)rem), dim3(GNT), 0, st, S.RB, Np, kb, kb + 1,
                               S.nblk, nzk);
        }
        if (rem > 1) {
            M2N_HIP(hipEventRecord(ev_fork, st));
            M2N_HIP(hipStreamWaitEvent(s2, ev_fork, 0));
            {
                M2N_PROF(ctx, s2, "k_syrk");
                hipLaunchKernelGGL(k_syrk, dim3((unsigned)((rem - 1) * rem / 2)), dim3(GNT), 0, s2, S.RB,
                                   Np, kb, kb + 2, S.nblk, nzk);
            }
            M2N_HIP(hipEventRecord(ev_join, s2));
        }
        potrf(kb + 1);
        if (rem > 1) {
            trsm(kb + 1);
            M2N_HIP(hipStreamWaitEvent(st, ev_join, 0));
        }
    }
    M2N_HIP(hipGetLastError());
    int hstatus = 0;
    M2N_HIP(hipMemcpyAsync(&hstatus, vst, sizeof(int), hipMemcpyDeviceToHost, st));
    M2N_HIP(hipStreamSynchronize(st));
    if (hstatus != 0) {
        set_error("R(B) is not numerically positive definite (Cholesky pivot %d)", -hstatus - 1);
        return M2N_ERR_NOT_PD;
    }
    return M2N_OK;
}

int gep_general(Ctx* ctx, hipStream_t st, const GepIn& g, const TStat& r) {
    const double* t_dev = g.t;
    const int64_t N = g.N;
    const double fmax = g.fmax, fw = g.fw;
    const int K = g.K;
    double* w_out = g.w;
    double* lambda_out = g.lambda;
    const double t0 = r.t0, tN = r.tN;
    const double cB = 2.0 * fmax;
    const bool lattice = on_lattice(g, r);
    const double span = N > 1 ? tN - t0 : 0.0;
    const double tc = 0.5 * (t0 + tN);
    const int Qn = quad_rank(fw, span, K);
    const bool lowrank = !lattice && Qn <= MAXP;
    Solver S;
    S.ctx = ctx;
    S.st = st;
    S.N = N;
    S.Np = (N + TB - 1) / TB * TB;
    S.K = K;
    S.lattice = lattice;
    const int64_t Np = S.Np;
    const int64_t nchunks = (Np + GRAM_ROWS - 1) / GRAM_ROWS;
    const int gram_wg = (int)(nchunks < GRAM_WG_MAX ? nchunks : GRAM_WG_MAX);
    const int cpw = (int)((nchunks + gram_wg - 1) / gram_wg);
    const int row_wg = (int)((Np + GNT - 1) / GNT);
    const int rot_wg = (int)((Np + 63) / 64);
    void *vY, *vpart, *vQ, *vth, *vgacc;
    M2N_TRY(ctx->workspace("gep_Q", sizeof(double) * MAXP * MAXP, &vQ));
    M2N_TRY(ctx->workspace("gep_th", sizeof(double) * MAXP, &vth));
    M2N_TRY(ctx->workspace("gep_gacc", sizeof(double) * 2 * MAXP * MAXP, &vgacc));
    double *Qm = (double*)vQ, *th = (double*)vth;
    double* gacc = (double*)vgacc;
    const double* td = t_dev;
    double* Y = nullptr;
    double* part = nullptr;
    auto need_Y = [&]() -> int {
        M2N_TRY(ctx->workspace("gep_Y", sizeof(double) * (size_t)MAXP * Np, &vY));
        M2N_TRY(ctx->workspace("gep_part", sizeof(double) * (size_t)row_wg * 2 * K + 64, &vpart));
        Y = (double*)vY;
        part = (double*)vpart;
        return M2N_OK;
    };

    // dense path: R(B) = L L^T by the tiled Cholesky (zero tiles skipped)
    auto factor_RB = [&]() -> int { return factor_dense(ctx, st, S, td, N, 0.0, fmax); };

    double scale;   // w = scale * (L^{-T}) y
    if (lowrank) {
        // ---- dense R(B): X = L^{-1} F with R(A0) = F F^T from the quadrature
        LrSeries d;
        std::memset(&d, 0, sizeof(d));
        d.t = t_dev;
        d.N = N;
        d.Np = Np;
        d.ldy = Np;
        d.tc = tc;
        d.span = span > 0.0 ? span : 1.0;
        d.fw = fw;
        d.scale = 1.0;
        d.c = 1.0;
        d.K = K;
        d.Qn = Qn;
        d.pF = Qn;
        d.nq = Qn / 2;
        d.fuse = 0;
        d.nchunks = (int)nchunks;
        d.nred = d.nchunks < 512 ? d.nchunks : 512;
        d.cpw = (d.nchunks + d.nred - 1) / d.nred;
        d.nred = (d.nchunks + d.cpw - 1) / d.cpw;
        M2N_TRY(gl_table(ctx, Qn, &d.glx));
        void *vF, *vgp;
        M2N_TRY(ctx->workspace("gep_F", sizeof(double) * (size_t)Qn * Np, &vF));
        M2N_TRY(ctx->workspace("gep_gpart", sizeof(double) * (size_t)d.nred * Qn * Qn, &vgp));
        d.F = (double*)vF;
        d.gpart = (double*)vgp;
        d.G = gacc;
        d.Z = Qm;
        d.theta = th;
        M2N_TRY(need_Y());
        d.Y = Y;
        {
            M2N_PROF(ctx, st, "k_lr_basis");
            dim3 gq((unsigned)((Np + 255) / 256), (unsigned)((d.nq + LR_QB - 1) / LR_QB), 1);
            hipLaunchKernelGGL(k_lr_basis, gq, dim3(256), 0, st, d, (const LrSeries*)nullptr);
        }
        M2N_HIP(hipGetLastError());
        M2N_TRY(factor_RB());
        S.p = Qn;
        M2N_TRY(S.trsv(d.F, 0));
        M2N_TRY(launch_gram_mfma(ctx, st, Qn, d.nred, 1, d, nullptr));
        {
            M2N_PROF(ctx, st, "k_sym_topk");
            launch_sym_topk(st, Qn, 1, d, nullptr);
        }
        M2N_TRY(launch_lr_expand(ctx, st, Qn, (Np + 63) / 64, 1, d, nullptr));
        M2N_HIP(hipGetLastError());
        S.p = K;
        M2N_TRY(S.trsv(Y, 1));   // w = L^{-T} y
        scale = std::sqrt(2.0 * fw);
    } else {
        // ---- wide band: block subspace iteration
        int p = (int)std::ceil(2.0 * fw * span) + 8;
        if (p < K + 8) p = K + 8;
        p = (p + 15) / 16 * 16;
        if (p > MAXP) p = MAXP;
        if (p > N) p = (int)N;
        S.p = p;
        void *vV, *vW, *vres;
        M2N_TRY(ctx->workspace("gep_V", sizeof(double) * (size_t)p * Np, &vV));
        M2N_TRY(ctx->workspace("gep_W", sizeof(double) * (size_t)p * Np, &vW));
        M2N_TRY(ctx->workspace("gep_res", sizeof(double) * (size_t)rot_wg * K, &vres));
        double *V = (double*)vV, *W = (double*)vW, *res = (double*)vres;
        M2N_TRY(need_Y());
        // W's padded rows are never written by the lattice convolution
        M2N_HIP(hipMemsetAsync(W, 0, sizeof(double) * (size_t)p * Np, st));
        if (lattice) {
            const int64_t Sspan = (int64_t)(tN - t0);
            int64_t M = 64;
            while (M < 2 * Sspan + 1) M *= 2;
            auto itp = ctx->fft64.find(M);
            if (itp == ctx->fft64.end()) {
                auto plan = std::make_unique<FftPlan64>();
                const int stp = make_fft64(ctx, M, *plan);
                if (stp != M2N_OK) {
                    release_fft(ctx, *plan);
                    return stp;
                }
                itp = ctx->fft64.emplace(M, std::move(plan)).first;
            }
            S.fft = itp->second.get();
            void *vmap, *vH, *vc1, *vc2, *vs;
            const int pairs = (p + 1) / 2;
            M2N_TRY(ctx->workspace("gep_map", sizeof(int) * (size_t)M, &vmap));
            M2N_TRY(ctx->workspace("gep_H", sizeof(double) * (size_t)M, &vH));
            M2N_TRY(ctx->workspace("gep_c1", sizeof(cplx<double>) * (size_t)M * pairs, &vc1));
            M2N_TRY(ctx->workspace("gep_c2", sizeof(cplx<double>) * (size_t)M * pairs, &vc2));
            M2N_TRY(ctx->workspace("gep_hs", sizeof(cplx<double>) * (size_t)M, &vs));
            S.map = (int*)vmap;
            S.Hhat = (double*)vH;
            S.cbuf1 = (cplx<double>*)vc1;
            S.cbuf2 = (cplx<double>*)vc2;
            {
                M2N_PROF(ctx, st, "k_lattice_setup");
                hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                                   S.map, M, -1);
                hipLaunchKernelGGL(k_lattice_map, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                                   td, N, S.map);
                hipLaunchKernelGGL(k_toep_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                                   S.cbuf2, M, Sspan, fw);
            }
            M2N_HIP(hipGetLastError());
            {
                M2N_PROF(ctx, st, "toeplitz_kernel_fft");
                ConvArgs a{};
                a.src = S.cbuf2;
                a.dst = S.cbuf1;
                M2N_TRY(run_fft64(*S.fft, st, a, 1, SRC_DIRECT, DST_DIRECT, (cplx<double>*)vs));
                hipLaunchKernelGGL(k_real_scale, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                                   (const cplx<double>*)S.cbuf1, M, 1.0 / ((double)M * cB), S.Hhat);
            }
            M2N_HIP(hipGetLastError());
            scale = std::sqrt(2.0 * fw / cB);
            M2N_TRY(subspace_solve(S, V, W, Y, gacc, res, Qm, th, nchunks));
        } else {
            M2N_TRY(factor_RB());
            void *vRA, *vtmp;
            M2N_TRY(ctx->workspace("gep_RA", sizeof(double) * (size_t)Np * Np, &vRA));
            M2N_TRY(ctx->workspace("gep_tmp", sizeof(double) * (size_t)p * Np, &vtmp));
            S.RA = (double*)vRA;
            S.tmp = (double*)vtmp;
            {
                M2N_PROF(ctx, st, "k_gen_sinc");
                dim3 gs((unsigned)((Np + 255) / 256), (unsigned)Np);
                hipLaunchKernelGGL(k_gen_sinc, gs, dim3(256), 0, st, td, N, Np, fw, 0.0, S.RA);
            }
            M2N_HIP(hipGetLastError());
            scale = std::sqrt(2.0 * fw);
            M2N_TRY(subspace_solve(S, V, W, Y, gacc, res, Qm, th, nchunks));
            M2N_TRY(S.trsv(Y, 1));   // w = L^{-T} y
        }
    }
    // ---- sign convention, scale, output
    {
        M2N_PROF(ctx, st, "k_sign_sums");
        hipLaunchKernelGGL(k_sign_sums, dim3(row_wg), dim3(GNT), 0, st, Y, Np, N, K, td, part);
    }
    {
        M2N_PROF(ctx, st, "k_finalize");
        const int fin_wg = (int)((N + GNT - 1) / GNT);
        hipLaunchKernelGGL(k_finalize, dim3(fin_wg), dim3(GNT), 0, st, Y, Np, N, K, scale, part,
                           row_wg, th, w_out, lambda_out);
    }
    M2N_HIP(hipGetLastError());
    M2N_HIP(hipStreamSynchronize(st));
    return M2N_OK;
}

int gep_run_batch(Ctx* ctx, hipStream_t st, const GepIn* in, int ns) {
    if (ns < 1 || !in) {
        set_error("empty batch");
        return M2N_ERR_ARG;
    }
    std::vector<TStat> stat;
    M2N_TRY(t_check(ctx, st, in, ns, stat));
    for (int i = 0; i < ns; ++i) M2N_TRY(t_status(stat[i], i));
    std::vector<int> lat, other;
    for (int i = 0; i < ns; ++i) (lattice_lowrank(in[i], stat[i]) ? lat : other).push_back(i);
    M2N_TRY(gep_lattice_batch(ctx, st, in, stat.data(), lat));
    for (int i : other) M2N_TRY(gep_general(ctx, st, in[i], stat[i]));
    return M2N_OK;
}

// One sub-band f_min <= |f| <= f_max with the nominal band |f - fc0| <= f_w:
// R(A0) w = lambda R(B^q) w (Sec. 2.4, Sec. 3.2) with complex tapers.
// R(B^q) = L L^T (real, dense); X = L^{-1} [Re(D F0) Im(D F0)] (2 Qn real
// columns); the complex Gram X^* X by k_herm_jacobi; y_k = X z_k / sqrt(theta_k)
// (real and imaginary parts as 2K real columns); w_k = sqrt(2 f_w) L^{-T} y_k
// (L is real) with the phase of k_finalize_c.  w is planar: real parts
// [K x N], then imaginary parts [K x N].
int gep_subband(Ctx* ctx, hipStream_t st, const double* t_dev, int64_t N, double fmin, double fmax,
                double fw, double fc0, int K, double* w_out, double* lambda_out) {
    GepIn g;
    g.t = t_dev;
    g.N = N;
    g.fmax = fmax;
    g.fw = fw;
    g.K = K;
    g.w = w_out;
    g.lambda = lambda_out;
    std::vector<TStat> stat;
    M2N_TRY(t_check(ctx, st, &g, 1, stat));
    M2N_TRY(t_status(stat[0], 0));
    const TStat& r = stat[0];
    const double span = N > 1 ? r.tN - r.t0 : 0.0;
    const int Qn = quad_rank(fw, span, K);
    if (2 * Qn > MAXP) {
        set_error("sub-band nominal band too wide for the complex low-rank path: quadrature rank %d "
                  "> %d (needs f_w (t_N - t_1) <= 4)", Qn, HQ);
        return M2N_ERR_UNSUPPORTED;
    }
    Solver S;
    S.ctx = ctx;
    S.st = st;
    S.N = N;
    S.Np = (N + TB - 1) / TB * TB;
    S.K = K;
    S.lattice = false;
    const int64_t Np = S.Np;
    const int64_t nchunks = (Np + GRAM_ROWS - 1) / GRAM_ROWS;
    const int row_wg = (int)((Np + GNT - 1) / GNT);
    LrSeries d;
    std::memset(&d, 0, sizeof(d));
    d.t = t_dev;
    d.N = N;
    d.Np = Np;
    d.ldy = Np;
    d.tc = 0.5 * (r.t0 + r.tN);
    d.span = span > 0.0 ? span : 1.0;
    d.fw = fw;
    d.scale = 1.0;
    d.c = 1.0;
    d.K = K;
    d.Qn = Qn;
    d.pF = 2 * Qn;
    d.nq = Qn / 2;
    d.fuse = 1;
    d.nchunks = (int)nchunks;
    d.nred = d.nchunks < 512 ? d.nchunks : 512;
    d.cpw = (d.nchunks + d.nred - 1) / d.nred;
    d.nred = (d.nchunks + d.cpw - 1) / d.cpw;
    M2N_TRY(gl_table(ctx, Qn, &d.glx));
    void *vF, *vgp, *vQ, *vth, *vgacc, *vY, *vpart;
    M2N_TRY(ctx->workspace("gep_F", sizeof(double) * (size_t)d.pF * Np, &vF));
    M2N_TRY(ctx->workspace("gep_gpart", sizeof(double) * (size_t)d.nred * d.pF * d.pF, &vgp));
    M2N_TRY(ctx->workspace("gep_Q", sizeof(double) * MAXP * MAXP, &vQ));
    M2N_TRY(ctx->workspace("gep_th", sizeof(double) * MAXP, &vth));
    M2N_TRY(ctx->workspace("gep_gacc", sizeof(double) * 2 * MAXP * MAXP, &vgacc));
    M2N_TRY(ctx->workspace("gep_Y", sizeof(double) * (size_t)MAXP * Np, &vY));
    M2N_TRY(ctx->workspace("gep_part", sizeof(double) * ((size_t)row_wg * 4 * K + 64), &vpart));
    d.F = (double*)vF;
    d.gpart = (double*)vgp;
    d.G = (double*)vgacc;
    d.Z = (double*)vQ;
    d.theta = (double*)vth;
    d.Y = (double*)vY;
    {
        M2N_PROF(ctx, st, "k_sb_basis");
        hipLaunchKernelGGL(k_sb_basis, dim3((unsigned)((Np + 255) / 256)), dim3(256), 0, st, d, fc0);
    }
    M2N_HIP(hipGetLastError());
    M2N_TRY(factor_dense(ctx, st, S, t_dev, N, fmin, fmax));
    S.p = 2 * Qn;
    M2N_TRY(S.trsv(d.F, 0));   // X = L^{-1} F
    M2N_TRY(launch_gram_mfma(ctx, st, d.pF, d.nred, 1, d, nullptr));
    {
        M2N_PROF(ctx, st, "k_herm_jacobi");
        hipLaunchKernelGGL(k_herm_jacobi, dim3(1), dim3(HJ_NT), 0, st, (const double*)d.G, Qn, K, d.theta, d.Z);
    }
    M2N_HIP(hipGetLastError());
    LrSeries e = d;   // the real expansion: 2 Qn columns into 2 K
    e.Qn = 2 * Qn;
    e.K = 2 * K;
    M2N_TRY(launch_lr_expand(ctx, st, e.Qn, (Np + 63) / 64, 1, e, nullptr));
    S.p = 2 * K;
    M2N_TRY(S.trsv(d.Y, 1));   // w = L^{-T} y
    {
        M2N_PROF(ctx, st, "k_phase_sums");
        hipLaunchKernelGGL(k_phase_sums, dim3(row_wg), dim3(GNT), 0, st, (const double*)d.Y, Np, N, K, t_dev,
                           fc0, (double*)vpart);
    }
    {
        M2N_PROF(ctx, st, "k_finalize_c");
        const int fin_wg = (int)((N + GNT - 1) / GNT);
        hipLaunchKernelGGL(k_finalize_c, dim3(fin_wg), dim3(GNT), 0, st, (const double*)d.Y, Np, N, K,
                           std::sqrt(2.0 * fw), (const double*)vpart, row_wg, (const double*)d.theta, w_out,
                           lambda_out);
    }
    M2N_HIP(hipGetLastError());
    M2N_HIP(hipStreamSynchronize(st));
    return M2N_OK;
}

int gep_run(Ctx* ctx, hipStream_t st, const double* t_dev, int64_t N, double fmax, double fw,
            int K, double* w_out, double* lambda_out) {
    GepIn g;
    g.t = t_dev;
    g.N = N;
    g.fmax = fmax;
    g.fw = fw;
    g.K = K;
    g.w = w_out;
    g.lambda = lambda_out;
    return gep_run_batch(ctx, st, &g, 1);
}

// The t check for callers outside this file: launched on `st`, `done`
// recorded after it; the summaries are read (after waiting for `done`) by the
// returned function.
int t_check_begin(Ctx* ctx, hipStream_t st, const double* const* t, const int64_t* N, int ns, hipEvent_t done,
                  std::function<void(std::vector<TSummary>&)>* read) {
    std::vector<GepIn> in((size_t)ns);
    for (int i = 0; i < ns; ++i) {
        in[i].t = t[i];
        in[i].N = N[i];
    }
    auto ds = std::make_shared<std::vector<TaSeries>>();
    M2N_TRY(t_check_launch(ctx, st, in.data(), ns, *ds));
    M2N_HIP(hipEventRecord(done, st));
    *read = [ds, done](std::vector<TSummary>& out) {
        (void)hipEventSynchronize(done);
        std::vector<TStat> r;
        t_check_read(*ds, r);
        out.assign(r.size(), TSummary());
        for (size_t i = 0; i < r.size(); ++i) {
            out[i].flags = r[i].flags;
            out[i].t0 = r[i].t0;
            out[i].tN = r[i].tN;
        }
    };
    return M2N_OK;
}

}  // namespace m2n
