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

// ------------------------------------------------------ Gram partials
// One pass over the rows of this workgroup's chunks:
//   part[wg][0 .. p*p)      = V^T V   (entry i * p + j)
//   part[wg][p*p .. 2 p*p)  = V^T W
__global__ __launch_bounds__(GNT) void k_gram2(const double* __restrict__ V, const double* __restrict__ W,
                                               int64_t Np, int64_t nrows, int p, int nchunks_per_wg,
                                               int64_t nchunks, double* __restrict__ part) {
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
            Ws[i][r] = in ? W[(int64_t)i * Np + r0 + r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + e * GNT;
            if (idx < 2 * np) {
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
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = threadIdx.x + e * GNT;
        if (idx < 2 * np) part[(int64_t)blockIdx.x * 2 * np + idx] = acc[e];
    }
}

// ------------------------------------- Rayleigh-Ritz on a general basis
// With G = V^T V = R^T R (Cholesky) and H = V^T W (W = C V), the Ritz pairs
// of C in span(V) are (theta, V Q) with Q = R^{-1} Q', where
// R^{-T} H R^{-1} = Q' diag(theta) Q'^T.  Y = V Q has orthonormal columns.
// The small symmetric eigenproblem is solved by parallel cyclic Jacobi:
// each round rotates n/2 disjoint index pairs (round-robin schedule).
// Output: Q (column-major, Q[i + j p] = component i of Ritz vector j) and
// theta, both in descending order of theta.
__global__ __launch_bounds__(GNT) void k_small_rr(const double* __restrict__ part, int nwg, int p,
                                                  double* __restrict__ Qout,
                                                  double* __restrict__ theta) {
    constexpr int LDA = MAXP + 1;
    __shared__ double G[MAXP * LDA];    // V^T V, then R (upper)
    __shared__ double H[MAXP * LDA];    // V^T W, then R^{-T} H R^{-1}, then Jacobi
    __shared__ double Qv[MAXP * LDA];   // Jacobi vectors
    __shared__ double cs[MAXP / 2][2];
    __shared__ int pr[MAXP / 2][2];
    __shared__ int order[MAXP];
    __shared__ double red[GNT / 64];
    __shared__ int s_any;
    const int tid = threadIdx.x;
    const int np = p * p;
    const int n = p + (p & 1);          // even size; a dummy index is decoupled
    // 1. sum the partials
    for (int e = tid; e < 2 * np; e += GNT) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int g = 0;
        for (; g + 3 < nwg; g += 4) {
            s0 += part[(int64_t)(g + 0) * 2 * np + e];
            s1 += part[(int64_t)(g + 1) * 2 * np + e];
            s2 += part[(int64_t)(g + 2) * 2 * np + e];
            s3 += part[(int64_t)(g + 3) * 2 * np + e];
        }
        for (; g < nwg; ++g) s0 += part[(int64_t)g * 2 * np + e];
        const double s = (s0 + s1) + (s2 + s3);
        const int q = e % np, i = q / p, j = q % p;
        if (e < np) G[i * LDA + j] = s;
        else H[i * LDA + j] = s;
    }
    __syncthreads();
    // symmetrise H
    for (int e = tid; e < np; e += GNT) {
        const int i = e / p, j = e % p;
        if (i < j) {
            const double m = 0.5 * (H[i * LDA + j] + H[j * LDA + i]);
            H[i * LDA + j] = m;
            H[j * LDA + i] = m;
        }
    }
    // 2. Cholesky G = R^T R (R upper, in place), pivots floored
    double dmax = 0.0;
    for (int i = 0; i < p; ++i) dmax = fmax(dmax, G[i * LDA + i]);
    const double pfloor = dmax * 1e-24 + 1e-300;
    for (int j = 0; j < p; ++j) {
        if (tid == 0) {
            const double d = G[j * LDA + j];
            G[j * LDA + j] = sqrt(d > pfloor ? d : pfloor);
        }
        __syncthreads();
        const double rjj = G[j * LDA + j];
        for (int c = j + 1 + tid; c < p; c += GNT) G[j * LDA + c] /= rjj;
        __syncthreads();
        const int rem = p - j - 1;
        for (int e = tid; e < rem * rem; e += GNT) {
            const int a = j + 1 + e / rem, b = j + 1 + e % rem;
            if (b >= a) G[a * LDA + b] -= G[j * LDA + a] * G[j * LDA + b];
        }
        __syncthreads();
    }
    // 3. H <- R^{-T} H  (forward substitution down each column)
    for (int c = tid; c < p; c += GNT) {
        for (int i = 0; i < p; ++i) {
            double s = H[i * LDA + c];
            for (int k = 0; k < i; ++k) s -= G[k * LDA + i] * H[k * LDA + c];
            H[i * LDA + c] = s / G[i * LDA + i];
        }
    }
    __syncthreads();
    //    H <- H R^{-1}  (forward substitution along each row)
    for (int r = tid; r < p; r += GNT) {
        for (int j = 0; j < p; ++j) {
            double s = H[r * LDA + j];
            for (int k = 0; k < j; ++k) s -= H[r * LDA + k] * G[k * LDA + j];
            H[r * LDA + j] = s / G[j * LDA + j];
        }
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += GNT) {
        const int i = e / n, j = e % n;
        if (i < p && j < p) {
            if (i < j) {
                const double m = 0.5 * (H[i * LDA + j] + H[j * LDA + i]);
                H[i * LDA + j] = m;
                H[j * LDA + i] = m;
            }
        } else {
            H[i * LDA + j] = (i == j) ? -1.0 : 0.0;   // dummy: decoupled, sorts last
        }
        Qv[i * LDA + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    // 4. parallel cyclic Jacobi
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) s_any = 0;
        __syncthreads();
        for (int r = 0; r < n - 1; ++r) {
            if (tid < n / 2) {
                int i, j;
                if (tid == 0) {
                    i = r;
                    j = n - 1;
                } else {
                    i = (r + tid) % (n - 1);
                    j = (r - tid + n - 1) % (n - 1);
                }
                if (i > j) {
                    const int tmp = i;
                    i = j;
                    j = tmp;
                }
                const double aij = H[i * LDA + j], aii = H[i * LDA + i], ajj = H[j * LDA + j];
                double c = 1.0, s = 0.0;
                if (fabs(aij) > 1e-18 * sqrt(fabs(aii * ajj)) && fabs(aij) > 1e-300) {
                    const double th = (ajj - aii) / (2.0 * aij);
                    double t = 1.0 / (fabs(th) + sqrt(th * th + 1.0));
                    if (th < 0.0) t = -t;
                    c = 1.0 / sqrt(t * t + 1.0);
                    s = t * c;
                    s_any = 1;
                }
                pr[tid][0] = i;
                pr[tid][1] = j;
                cs[tid][0] = c;
                cs[tid][1] = s;
            }
            __syncthreads();
            // rows i, j of H  <- J^T H
            for (int e = tid; e < (n / 2) * n; e += GNT) {
                const int k = e / n, m = e % n;
                const double s = cs[k][1];
                if (s != 0.0) {
                    const int i = pr[k][0], j = pr[k][1];
                    const double c = cs[k][0];
                    const double hi = H[i * LDA + m], hj = H[j * LDA + m];
                    H[i * LDA + m] = c * hi - s * hj;
                    H[j * LDA + m] = s * hi + c * hj;
                }
            }
            __syncthreads();
            // columns i, j of H and of Q  <- H J, Q J
            for (int e = tid; e < (n / 2) * n; e += GNT) {
                const int k = e / n, m = e % n;
                const double s = cs[k][1];
                if (s != 0.0) {
                    const int i = pr[k][0], j = pr[k][1];
                    const double c = cs[k][0];
                    const double hi = H[m * LDA + i], hj = H[m * LDA + j];
                    H[m * LDA + i] = c * hi - s * hj;
                    H[m * LDA + j] = s * hi + c * hj;
                    const double qi = Qv[m * LDA + i], qj = Qv[m * LDA + j];
                    Qv[m * LDA + i] = c * qi - s * qj;
                    Qv[m * LDA + j] = s * qi + c * qj;
                }
            }
            __syncthreads();
        }
        if (!s_any) break;
    }
    // 5. order by descending eigenvalue (dummy last)
    if (tid == 0) {
        for (int i = 0; i < n; ++i) order[i] = i;
        for (int i = 0; i < n; ++i) {
            int best = i;
            for (int j = i + 1; j < n; ++j)
                if (H[order[j] * LDA + order[j]] > H[order[best] * LDA + order[best]]) best = j;
            const int tmp = order[i];
            order[i] = order[best];
            order[best] = tmp;
        }
    }
    __syncthreads();
    // 6. Q = R^{-1} Q'  (back substitution down each kept column)
    for (int jc = tid; jc < p; jc += GNT) {
        const int src = order[jc];
        double x[MAXP];
        for (int i = p - 1; i >= 0; --i) {
            double s = Qv[i * LDA + src];
            for (int k = i + 1; k < p; ++k) s -= G[i * LDA + k] * x[k];
            x[i] = s / G[i * LDA + i];
        }
        for (int i = 0; i < p; ++i) Qout[i + jc * p] = x[i];
        theta[jc] = H[src * LDA + src];
    }
    (void)red;
}

// ---------------------------------- Ritz vectors, next block, residuals
// Y = V Q (orthonormal Ritz vectors), Z = W Q = C Y;
//   res[wg][k] = sum_n (Z_nk - theta_k Y_nk)^2        (k < K)
//   V <- Z diag(1 / max(theta, floor))  (next block; in place)
// Rows >= N are zero.  PC is p rounded up to a multiple of 8.
template <int PC>
__global__ __launch_bounds__(GNT) void k_rotate2(double* __restrict__ V, const double* __restrict__ W,
                                                 const double* __restrict__ Q,
                                                 const double* __restrict__ theta, int64_t Np,
                                                 int64_t N, int p, int K, double* __restrict__ Y,
                                                 double* __restrict__ res) {
    __shared__ double Qs[PC * PC];
    __shared__ double th[PC];
    __shared__ double red[PC];
    for (int e = threadIdx.x; e < PC * PC; e += GNT) {
        const int i = e % PC, j = e / PC;
        Qs[e] = (i < p && j < p) ? Q[i + j * p] : 0.0;
    }
    for (int e = threadIdx.x; e < PC; e += GNT) {
        th[e] = e < p ? theta[e] : 1.0;
        red[e] = 0.0;
    }
    __syncthreads();
    const double floor_t = fabs(th[0]) * 1e-6 + 1e-300;
    const int64_t n = (int64_t)blockIdx.x * GNT + threadIdx.x;
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
                if (j < K) {
                    const double d = z - tj * y;
                    atomicAdd(&red[j], d * d);
                }
            }
        }
    } else if (n < Np) {
        for (int j = 0; j < p; ++j) {
            Y[(int64_t)j * Np + n] = 0.0;
            V[(int64_t)j * Np + n] = 0.0;
        }
    }
    __syncthreads();
    if (threadIdx.x < K) res[(int64_t)blockIdx.x * K + threadIdx.x] = red[threadIdx.x];
}

// ------------------------------------------------------ lattice helpers
__global__ void k_fill_int(int* __restrict__ a, int64_t n, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_lattice_map(const int* __restrict__ off, int64_t N, int* __restrict__ map) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) map[off[n]] = (int)n;
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

// Cholesky of the TB x TB diagonal block kb (in place, lower; upper zeroed)
__global__ __launch_bounds__(GNT) void k_potrf(double* __restrict__ A, int64_t Np, int kb, int64_t N,
                                               int* __restrict__ status) {
    __shared__ double T[TB][TB + 1];
    const int64_t o = (int64_t)kb * TB;
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int i = e % TB, j = e / TB;
        T[i][j] = A[(o + i) + (o + j) * Np];
    }
    __syncthreads();
    for (int j = 0; j < TB; ++j) {
        if (threadIdx.x == 0) {
            const double d = T[j][j];
            if (!(d > 0.0)) {
                if (o + j < N) atomicCAS(status, 0, -(int)(o + j + 1));
                T[j][j] = 1.0;   // keep going; the status reports the failure
            } else {
                T[j][j] = sqrt(d);
            }
        }
        __syncthreads();
        for (int i = j + 1 + threadIdx.x; i < TB; i += GNT) T[i][j] /= T[j][j];
        __syncthreads();
        const int rem = TB - j - 1;
        for (int e = threadIdx.x; e < rem * rem; e += GNT) {
            const int i = j + 1 + e % rem, k = j + 1 + e / rem;
            if (i >= k) T[i][k] -= T[i][j] * T[k][j];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int i = e % TB, j = e / TB;
        A[(o + i) + (o + j) * Np] = (i >= j) ? T[i][j] : 0.0;
    }
}

// panel: A_ik <- A_ik L_kk^{-T} for row blocks i > kb; nz[i] = tile not all zero
__global__ __launch_bounds__(GNT) void k_trsm_panel(double* __restrict__ A, int64_t Np, int kb,
                                                    int* __restrict__ nz) {
    __shared__ double L[TB][TB + 1];
    __shared__ double X[TB][TB + 1];
    __shared__ int any;
    const int ib = kb + 1 + blockIdx.x;
    const int64_t o = (int64_t)kb * TB, r = (int64_t)ib * TB;
    if (threadIdx.x == 0) any = 0;
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int i = e % TB, j = e / TB;
        L[i][j] = A[(o + i) + (o + j) * Np];
        X[i][j] = A[(r + i) + (o + j) * Np];
    }
    __syncthreads();
    // row i of X solves x L^T = a: x_c = (a_c - sum_{j<c} x_j L_cj) / L_cc
    if (threadIdx.x < TB) {
        const int i = threadIdx.x;
        int mine = 0;
        for (int c = 0; c < TB; ++c) {
            double s = X[i][c];
            for (int j = 0; j < c; ++j) s -= X[i][j] * L[c][j];
            s /= L[c][c];
            X[i][c] = s;
            mine |= (s != 0.0);
        }
        if (mine) atomicOr(&any, 1);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int i = e % TB, j = e / TB;
        A[(r + i) + (o + j) * Np] = X[i][j];
    }
    if (threadIdx.x == 0) nz[ib] = any;
}

// trailing update A_ij -= L_ik L_jk^T over lower tiles kb < jb <= ib,
// skipped when either panel tile is exactly zero
__global__ __launch_bounds__(GNT) void k_syrk(double* __restrict__ A, int64_t Np, int kb, int nblk,
                                              const int* __restrict__ nz) {
    __shared__ double Li[TB][TB + 1];
    __shared__ double Lj[TB][TB + 1];
    // map blockIdx.x to (ib, jb) with kb < jb <= ib < nblk
    const int m = nblk - kb - 1;
    int idx = blockIdx.x, jj = 0;
    while (idx >= m - jj) {
        idx -= m - jj;
        ++jj;
    }
    const int jb = kb + 1 + jj, ib = jb + idx;
    if (!nz[ib] || !nz[jb]) return;
    const int64_t o = (int64_t)kb * TB, ri = (int64_t)ib * TB, rj = (int64_t)jb * TB;
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int i = e % TB, k = e / TB;
        Li[i][k] = A[(ri + i) + (o + k) * Np];
        Lj[i][k] = A[(rj + i) + (o + k) * Np];
    }
    __syncthreads();
    // thread owns a 4 x 4 sub-tile
    const int tr = (threadIdx.x % 16) * 4, tc = (threadIdx.x / 16) * 4;
    double acc[4][4] = {};
    for (int k = 0; k < TB; ++k) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = Li[tr + u][k];
            b[u] = Lj[tc + u][k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t gi = ri + tr + u, gj = rj + tc + v;
            if (ib != jb || gi >= gj) A[gi + gj * Np] -= acc[u][v];
        }
}

// triangular solve with one TB x TB diagonal block for p columns:
//   lower (trans = 0):  L_kk X = B_k;   upper (trans = 1): L_kk^T X = B_k
__global__ __launch_bounds__(GNT) void k_trsv_diag(const double* __restrict__ A, int64_t Np, int kb,
                                                   int trans, double* __restrict__ Bm, int p) {
    __shared__ double L[TB][TB + 1];
    const int64_t o = (int64_t)kb * TB;
    for (int e = threadIdx.x; e < TB * TB; e += GNT) {
        const int i = e % TB, j = e / TB;
        L[i][j] = A[(o + i) + (o + j) * Np];
    }
    __syncthreads();
    const int col = threadIdx.x;
    if (col >= p) return;
    double x[TB];
    double* bcol = Bm + (int64_t)col * Np + o;
    for (int i = 0; i < TB; ++i) x[i] = bcol[i];
    if (!trans) {
        for (int i = 0; i < TB; ++i) {
            double s = x[i];
            for (int j = 0; j < i; ++j) s -= L[i][j] * x[j];
            x[i] = s / L[i][i];
        }
    } else {
        for (int i = TB - 1; i >= 0; --i) {
            double s = x[i];
            for (int j = i + 1; j < TB; ++j) s -= L[j][i] * x[j];
            x[i] = s / L[i][i];
        }
    }
    for (int i = 0; i < TB; ++i) bcol[i] = x[i];
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

// ------------------------------------------------------------ host side
struct FftPlan64 {
    int64_t M = 0;
    int log_M = 0;
    bool single = false;
    int N1 = 0, N2 = 0, BB = 0, MM = 0, lo_bits = 0, tw_len = 0;
    DevBuf tw, tw_lo, tw_hi;
};

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
    FftPlan64 fft;
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
            if (fft.single) {
                // whole convolution in two single-workgroup transforms
                a.dst = cbuf1;
                M2N_TRY(run_fft64(fft, st, a, pairs, SRC_PAIR, DST_MULCONJ, nullptr));
                a.src = cbuf1;
                M2N_TRY(run_fft64(fft, st, a, pairs, SRC_DIRECT, DST_PAIR, nullptr));
            } else {
                a.dst = cbuf1;
                M2N_TRY(run_fft64(fft, st, a, pairs, SRC_PAIR, DST_MULCONJ, cbuf2));
                a.src = cbuf1;
                M2N_TRY(run_fft64(fft, st, a, pairs, SRC_DIRECT, DST_PAIR, cbuf2));
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
                hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(GNT), 0, st, RB, Np, kb, trans, Bm, p);
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
int subspace_solve(Solver& S, double* V, double* W, double* Y, double* part, double* res,
                   double* Q, double* th, int64_t nchunks) {
    Ctx* ctx = S.ctx;
    hipStream_t st = S.st;
    const int64_t N = S.N, Np = S.Np;
    const int p = S.p, K = S.K;
    const int gram_wg = (int)(nchunks < 32 ? nchunks : 32);
    const int cpw = (int)((nchunks + gram_wg - 1) / gram_wg);
    const int row_wg = (int)((Np + GNT - 1) / GNT);
    const int pc = (p + 7) / 8 * 8;
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
                               part);
        }
        {
            M2N_PROF(ctx, st, "k_small_rr");
            hipLaunchKernelGGL(k_small_rr, dim3(1), dim3(GNT), 0, st, part, gram_wg, p, Q, th);
        }
        {
            M2N_PROF(ctx, st, "k_rotate2");
#define M2N_ROT(PCV)                                                                            \
    case PCV:                                                                                   \
        hipLaunchKernelGGL(k_rotate2<PCV>, dim3(row_wg), dim3(GNT), 0, st, V, W, Q, th, Np, N, p, \
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

int gep_run(Ctx* ctx, hipStream_t st, const double* t_dev, int64_t N, double fmax, double fw,
            int K, double* w_out, double* lambda_out) {
    // ---- host analysis of the sampling times
    std::vector<double> t(N);
    M2N_HIP(hipMemcpyAsync(t.data(), t_dev, sizeof(double) * (size_t)N, hipMemcpyDeviceToHost, st));
    M2N_HIP(hipStreamSynchronize(st));
    bool integral = true;
    for (int64_t n = 0; n < N; ++n) {
        if (!std::isfinite(t[n])) {
            set_error("non-finite sampling time at %lld", (long long)n);
            return M2N_ERR_ARG;
        }
        if (n > 0 && !(t[n] > t[n - 1])) {
            set_error("sampling times not strictly increasing at %lld", (long long)n);
            return M2N_ERR_T_ORDER;
        }
        if (t[n] != std::rint(t[n]) || std::fabs(t[n]) > 4.0e15) integral = false;
    }
    const double cB = 2.0 * fmax;
    const bool lattice = integral && cB == std::rint(cB) && cB >= 1.0 && (t[N - 1] - t[0]) < 2.0e6;
    const double span = N > 1 ? t[N - 1] - t[0] : 0.0;
    int p = (int)std::ceil(2.0 * fw * span) + 8;
    if (p < K + 8) p = K + 8;
    p = (p + 15) / 16 * 16;
    if (p > MAXP) p = MAXP;
    if (p > N) p = (int)N;
    if (p < K) {
        set_error("internal: block width %d < K %d", p, K);
        return M2N_ERR_ARG;
    }
    Solver S;
    S.ctx = ctx;
    S.st = st;
    S.N = N;
    S.Np = (N + TB - 1) / TB * TB;
    S.p = p;
    S.K = K;
    S.lattice = lattice;
    const int64_t Np = S.Np;
    const int64_t nchunks = (Np + GRAM_ROWS - 1) / GRAM_ROWS;
    const int row_wg = (int)((Np + GNT - 1) / GNT);
    void *vV, *vW, *vY, *vpart, *vres, *vQ, *vth, *vt;
    M2N_TRY(ctx->workspace("gep_V", sizeof(double) * (size_t)p * Np, &vV));
    M2N_TRY(ctx->workspace("gep_W", sizeof(double) * (size_t)p * Np, &vW));
    M2N_TRY(ctx->workspace("gep_Y", sizeof(double) * (size_t)p * Np, &vY));
    size_t part_n = (size_t)32 * 2 * p * p;
    if (part_n < (size_t)row_wg * 2 * K) part_n = (size_t)row_wg * 2 * K;
    M2N_TRY(ctx->workspace("gep_part", sizeof(double) * part_n, &vpart));
    M2N_TRY(ctx->workspace("gep_res", sizeof(double) * (size_t)row_wg * K, &vres));
    M2N_TRY(ctx->workspace("gep_Q", sizeof(double) * MAXP * MAXP, &vQ));
    M2N_TRY(ctx->workspace("gep_th", sizeof(double) * MAXP, &vth));
    M2N_TRY(ctx->workspace("gep_t", sizeof(double) * (size_t)N, &vt));
    double *V = (double*)vV, *W = (double*)vW, *Y = (double*)vY;
    double *part = (double*)vpart, *res = (double*)vres, *Q = (double*)vQ, *th = (double*)vth;
    M2N_HIP(hipMemcpyAsync(vt, t_dev, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, st));
    const double* td = (const double*)vt;
    // W's padded rows are never written by the lattice convolution
    M2N_HIP(hipMemsetAsync(W, 0, sizeof(double) * (size_t)p * Np, st));

    double scale;   // w = scale * (L^{-T}) y
    if (lattice) {
        // ---- lattice: R(B) = cB I, C = R(A0) / cB
        const int64_t Sspan = (int64_t)(t[N - 1] - t[0]);
        int64_t M = 64;
        while (M < 2 * Sspan + 1) M *= 2;
        M2N_TRY(make_fft64(ctx, M, S.fft));
        struct Guard {
            Ctx* c;
            FftPlan64* f;
            ~Guard() { release_fft(c, *f); }
        } guard{ctx, &S.fft};
        std::vector<int> off(N);
        for (int64_t n = 0; n < N; ++n) off[n] = (int)(t[n] - t[0]);
        void *vmap, *voff, *vH, *vc1, *vc2, *vs;
        const int pairs = (p + 1) / 2;
        M2N_TRY(ctx->workspace("gep_map", sizeof(int) * (size_t)M, &vmap));
        M2N_TRY(ctx->workspace("gep_off", sizeof(int) * (size_t)N, &voff));
        M2N_TRY(ctx->workspace("gep_H", sizeof(double) * (size_t)M, &vH));
        M2N_TRY(ctx->workspace("gep_c1", sizeof(cplx<double>) * (size_t)M * pairs, &vc1));
        M2N_TRY(ctx->workspace("gep_c2", sizeof(cplx<double>) * (size_t)M * pairs, &vc2));
        M2N_TRY(ctx->workspace("gep_hs", sizeof(cplx<double>) * (size_t)M, &vs));
        M2N_HIP(hipMemcpyAsync(voff, off.data(), sizeof(int) * (size_t)N, hipMemcpyHostToDevice, st));
        S.map = (int*)vmap;
        S.Hhat = (double*)vH;
        S.cbuf1 = (cplx<double>*)vc1;
        S.cbuf2 = (cplx<double>*)vc2;
        {
            M2N_PROF(ctx, st, "k_lattice_setup");
            hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, S.map,
                               M, -1);
            hipLaunchKernelGGL(k_lattice_map, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                               (const int*)voff, N, S.map);
            // Hhat = FFT(h) / (M cB)
            hipLaunchKernelGGL(k_toep_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                               S.cbuf2, M, Sspan, fw);
        }
        M2N_HIP(hipGetLastError());
        {
            M2N_PROF(ctx, st, "toeplitz_kernel_fft");
            ConvArgs a{};
            a.src = S.cbuf2;
            a.dst = S.cbuf1;
            M2N_TRY(run_fft64(S.fft, st, a, 1, SRC_DIRECT, DST_DIRECT, (cplx<double>*)vs));
            hipLaunchKernelGGL(k_real_scale, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                               (const cplx<double>*)S.cbuf1, M, 1.0 / ((double)M * cB), S.Hhat);
        }
        M2N_HIP(hipGetLastError());
        scale = std::sqrt(2.0 * fw / cB);
        M2N_TRY(subspace_solve(S, V, W, Y, part, res, Q, th, nchunks));
    } else {
        // ---- dense: R(B) = L L^T, C = L^{-1} R(A0) L^{-T}
        if (Np > 65536) {
            set_error("dense GEP limited to N <= 65536 in this build");
            return M2N_ERR_UNSUPPORTED;
        }
        S.nblk = (int)(Np / TB);
        void *vRB, *vRA, *vtmp, *vnz, *vst;
        M2N_TRY(ctx->workspace("gep_RB", sizeof(double) * (size_t)Np * Np, &vRB));
        M2N_TRY(ctx->workspace("gep_RA", sizeof(double) * (size_t)Np * Np, &vRA));
        M2N_TRY(ctx->workspace("gep_tmp", sizeof(double) * (size_t)p * Np, &vtmp));
        M2N_TRY(ctx->workspace("gep_nz", sizeof(int) * (size_t)S.nblk, &vnz));
        M2N_TRY(ctx->workspace("gep_status", 64, &vst));
        S.RB = (double*)vRB;
        S.RA = (double*)vRA;
        S.tmp = (double*)vtmp;
        S.nz = (int*)vnz;
        M2N_HIP(hipMemsetAsync(vst, 0, 64, st));
        {
            M2N_PROF(ctx, st, "k_gen_sinc");
            dim3 gs((unsigned)((Np + 255) / 256), (unsigned)Np);
            hipLaunchKernelGGL(k_gen_sinc, gs, dim3(256), 0, st, td, N, Np, fmax, 1.0, S.RB);
            hipLaunchKernelGGL(k_gen_sinc, gs, dim3(256), 0, st, td, N, Np, fw, 0.0, S.RA);
        }
        M2N_HIP(hipGetLastError());
        for (int kb = 0; kb < S.nblk; ++kb) {
            {
                M2N_PROF(ctx, st, "k_potrf");
                hipLaunchKernelGGL(k_potrf, dim3(1), dim3(GNT), 0, st, S.RB, Np, kb, N, (int*)vst);
            }
            const int rem = S.nblk - kb - 1;
            if (rem > 0) {
                {
                    M2N_PROF(ctx, st, "k_trsm_panel");
                    hipLaunchKernelGGL(k_trsm_panel, dim3(rem), dim3(GNT), 0, st, S.RB, Np, kb, S.nz);
                }
                const int ntiles = rem * (rem + 1) / 2;
                M2N_PROF(ctx, st, "k_syrk");
                hipLaunchKernelGGL(k_syrk, dim3(ntiles), dim3(GNT), 0, st, S.RB, Np, kb, S.nblk, S.nz);
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
        scale = std::sqrt(2.0 * fw);
        M2N_TRY(subspace_solve(S, V, W, Y, part, res, Q, th, nchunks));
        // y -> L^{-T} y
        M2N_TRY(S.trsv(Y, 1));
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

}  // namespace m2n
