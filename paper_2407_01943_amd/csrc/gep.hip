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
// part[wg][i * pb + j] = sum over this workgroup's rows of A[i][n] * B[j][n]
__global__ __launch_bounds__(GNT) void k_gram(const double* __restrict__ A, const double* __restrict__ B,
                                              int64_t Np, int64_t nrows, int pa, int pb, int nchunks_per_wg,
                                              int64_t nchunks, double* __restrict__ part) {
    __shared__ double As[MAXP][GRAM_ROWS + 1];
    __shared__ double Bs[MAXP][GRAM_ROWS + 1];
    const int np = pa * pb;
    double acc[MAXP * MAXP / GNT];
    constexpr int PER = MAXP * MAXP / GNT;
#pragma unroll
    for (int e = 0; e < PER; ++e) acc[e] = 0.0;
    const int64_t c0 = (int64_t)blockIdx.x * nchunks_per_wg;
    for (int64_t c = c0; c < c0 + nchunks_per_wg && c < nchunks; ++c) {
        const int64_t r0 = c * GRAM_ROWS;
        for (int e = threadIdx.x; e < pa * GRAM_ROWS; e += GNT) {
            const int i = e / GRAM_ROWS, r = e % GRAM_ROWS;
            As[i][r] = (r0 + r < nrows) ? A[(int64_t)i * Np + r0 + r] : 0.0;
        }
        for (int e = threadIdx.x; e < pb * GRAM_ROWS; e += GNT) {
            const int i = e / GRAM_ROWS, r = e % GRAM_ROWS;
            Bs[i][r] = (r0 + r < nrows) ? B[(int64_t)i * Np + r0 + r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + e * GNT;
            if (idx < np) {
                const int i = idx / pb, j = idx % pb;
                double s = 0.0;
                for (int r = 0; r < GRAM_ROWS; ++r) s += As[i][r] * Bs[j][r];
                acc[e] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = threadIdx.x + e * GNT;
        if (idx < np) part[(int64_t)blockIdx.x * np + idx] = acc[e];
    }
}

// ------------------------------------------- Rayleigh-Ritz: sum + Jacobi
// H = sum of the Gram partials (p x p, symmetrised), then cyclic Jacobi in
// LDS; Q (column-major, Q[i + j p] = component i of eigenvector j) and theta
// sorted in descending order.
__global__ __launch_bounds__(64) void k_rr(const double* __restrict__ part, int nwg, int p,
                                           double* __restrict__ Q, double* __restrict__ theta) {
    __shared__ double A[MAXP][MAXP + 1];
    __shared__ double Vv[MAXP][MAXP + 1];
    __shared__ double rot[4];
    __shared__ double sred[64];
    __shared__ int order[MAXP];
    const int lane = threadIdx.x;
    for (int e = lane; e < p * p; e += 64) {
        double s = 0.0;
        for (int g = 0; g < nwg; ++g) s += part[(int64_t)g * p * p + e];
        A[e / p][e % p] = s;
    }
    __syncthreads();
    for (int e = lane; e < p * p; e += 64) {
        const int i = e / p, j = e % p;
        if (i < j) {
            const double m = 0.5 * (A[i][j] + A[j][i]);
            A[i][j] = m;
            A[j][i] = m;
        }
        Vv[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, fro = 0.0;
        for (int e = lane; e < p * p; e += 64) {
            const int i = e / p, j = e % p;
            const double v = A[i][j] * A[i][j];
            fro += v;
            if (i != j) off += v;
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o, 64);
            fro += __shfl_xor(fro, o, 64);
        }
        if (off <= 1e-30 * fro || off == 0.0) break;
        for (int i = 0; i < p - 1; ++i) {
            for (int j = i + 1; j < p; ++j) {
                if (lane == 0) {
                    const double aij = A[i][j];
                    double c = 1.0, s = 0.0, t = 0.0, tau = 0.0;
                    if (aij != 0.0 && fabs(aij) > 1e-300) {
                        const double th = (A[j][j] - A[i][i]) / (2.0 * aij);
                        t = 1.0 / (fabs(th) + sqrt(th * th + 1.0));
                        if (th < 0.0) t = -t;
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                        tau = s / (1.0 + c);
                    }
                    rot[0] = s;
                    rot[1] = tau;
                    rot[2] = t;
                    rot[3] = aij;
                }
                __syncthreads();
                const double s = rot[0], tau = rot[1], t = rot[2], aij = rot[3];
                if (s != 0.0) {
                    for (int m = lane; m < p; m += 64) {
                        if (m != i && m != j) {
                            const double ami = A[m][i], amj = A[m][j];
                            const double ni = ami - s * (amj + tau * ami);
                            const double nj = amj + s * (ami - tau * amj);
                            A[m][i] = ni;
                            A[i][m] = ni;
                            A[m][j] = nj;
                            A[j][m] = nj;
                        }
                        const double vmi = Vv[m][i], vmj = Vv[m][j];
                        Vv[m][i] = vmi - s * (vmj + tau * vmi);
                        Vv[m][j] = vmj + s * (vmi - tau * vmj);
                    }
                    __syncthreads();
                    if (lane == 0) {
                        A[i][i] -= t * aij;
                        A[j][j] += t * aij;
                        A[i][j] = 0.0;
                        A[j][i] = 0.0;
                    }
                }
                __syncthreads();
            }
        }
    }
    // sort descending (lane 0, p <= 64)
    if (lane == 0) {
        for (int i = 0; i < p; ++i) order[i] = i;
        for (int i = 0; i < p; ++i) {
            int best = i;
            for (int j = i + 1; j < p; ++j)
                if (A[order[j]][order[j]] > A[order[best]][order[best]]) best = j;
            const int tmp = order[i];
            order[i] = order[best];
            order[best] = tmp;
        }
    }
    __syncthreads();
    for (int e = lane; e < p * p; e += 64) {
        const int i = e % p, j = e / p;   // component i of eigenvector j
        Q[e] = Vv[i][order[j]];
    }
    for (int j = lane; j < p; j += 64) theta[j] = A[order[j]][order[j]];
    (void)sred;
}

// ---------------------------------- Ritz vectors, next block, residuals
// Y = V Q, U = (W Q) / max(theta, floor), residual partials for the first K:
//   res[wg][k] = sum_n ((W Q)_{nk} - theta_k (V Q)_{nk})^2
__global__ __launch_bounds__(GNT) void k_rotate(const double* __restrict__ V, const double* __restrict__ W,
                                                const double* __restrict__ Q,
                                                const double* __restrict__ theta, int64_t Np,
                                                int64_t N, int p, int K, double* __restrict__ Y,
                                                double* __restrict__ U, double* __restrict__ res) {
    __shared__ double Qs[MAXP * MAXP];
    __shared__ double th[MAXP];
    __shared__ double red[GNT / 64][MAXP];
    for (int e = threadIdx.x; e < p * p; e += GNT) Qs[e] = Q[e];
    for (int e = threadIdx.x; e < p; e += GNT) th[e] = theta[e];
    __syncthreads();
    const double floor_t = fabs(th[0]) * 1e-13 + 1e-300;
    const int64_t n = (int64_t)blockIdx.x * GNT + threadIdx.x;
    double rk[MAXP];
#pragma unroll
    for (int k = 0; k < MAXP; ++k) rk[k] = 0.0;
    if (n >= N && n < Np) {
        for (int j = 0; j < p; ++j) {
            Y[(int64_t)j * Np + n] = 0.0;
            U[(int64_t)j * Np + n] = 0.0;
        }
    } else if (n < N) {
        for (int j = 0; j < p; ++j) {
            double y = 0.0, u = 0.0;
            for (int i = 0; i < p; ++i) {
                const double q = Qs[j * p + i];
                y += V[(int64_t)i * Np + n] * q;
                u += W[(int64_t)i * Np + n] * q;
            }
            Y[(int64_t)j * Np + n] = y;
            const double tj = th[j];
            U[(int64_t)j * Np + n] = u / (fabs(tj) > floor_t ? tj : floor_t);
            if (j < K) {
                const double d = u - tj * y;
                rk[j] = d * d;
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < K; ++k) {
        double v = rk[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int w = 0; w < GNT / 64; ++w) s += red[w][threadIdx.x];
        res[(int64_t)blockIdx.x * K + threadIdx.x] = s;
    }
}

// ------------------------------------------------------------- CholQR
// G = sum of Gram partials; upper R with G = R^T R (pivot floored so a
// dependent column is re-normalised instead of dividing by zero).
__global__ __launch_bounds__(64) void k_chol_small(const double* __restrict__ part, int nwg, int p,
                                                   double* __restrict__ Rout) {
    __shared__ double G[MAXP][MAXP + 1];
    const int lane = threadIdx.x;
    for (int e = lane; e < p * p; e += 64) {
        double s = 0.0;
        for (int g = 0; g < nwg; ++g) s += part[(int64_t)g * p * p + e];
        G[e / p][e % p] = s;
    }
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < p; ++i) dmax = fmax(dmax, G[i][i]);
    const double floor_p = dmax * 1e-28 + 1e-300;
    for (int j = 0; j < p; ++j) {
        if (lane == 0) {
            double d = G[j][j];
            for (int k = 0; k < j; ++k) d -= G[k][j] * G[k][j];
            G[j][j] = sqrt(d > floor_p ? d : floor_p);
        }
        __syncthreads();
        for (int c = j + 1 + lane; c < p; c += 64) {
            double s = G[j][c];
            for (int k = 0; k < j; ++k) s -= G[k][j] * G[k][c];
            G[j][c] = s / G[j][j];
        }
        __syncthreads();
    }
    for (int e = lane; e < p * p; e += 64) {
        const int i = e / p, j = e % p;   // R[i][j], upper
        Rout[e] = (j >= i) ? G[i][j] : 0.0;
    }
}

// V = U R^{-1}, row by row:  v_j = (u_j - sum_{i<j} v_i R_ij) / R_jj
__global__ __launch_bounds__(GNT) void k_trsm_rows(const double* __restrict__ U, const double* __restrict__ Rm,
                                                   int64_t Np, int64_t N, int p, double* __restrict__ V) {
    __shared__ double Rs[MAXP * MAXP];
    for (int e = threadIdx.x; e < p * p; e += GNT) Rs[e] = Rm[e];
    __syncthreads();
    const int64_t n = (int64_t)blockIdx.x * GNT + threadIdx.x;
    if (n >= Np) return;
    double v[MAXP];
    for (int j = 0; j < p; ++j) {
        double s = n < N ? U[(int64_t)j * Np + n] : 0.0;
        for (int i = 0; i < j; ++i) s -= v[i] * Rs[i * p + j];
        v[j] = s / Rs[j * p + j];
        V[(int64_t)j * Np + n] = v[j];
    }
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
    const bool lattice = integral && cB == std::rint(cB) && cB >= 1.0 &&
                         (t[N - 1] - t[0]) < 2.0e6;
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
    void *vV, *vW, *vU, *vY, *vpart, *vres, *vQ, *vth, *vR;
    const int64_t nchunks = (Np + GRAM_ROWS - 1) / GRAM_ROWS;
    const int gram_wg = (int)(nchunks < 120 ? nchunks : 120);
    const int cpw = (int)((nchunks + gram_wg - 1) / gram_wg);
    const int row_wg = (int)((Np + GNT - 1) / GNT);
    M2N_TRY(ctx->workspace("gep_V", sizeof(double) * (size_t)p * Np, &vV));
    M2N_TRY(ctx->workspace("gep_W", sizeof(double) * (size_t)p * Np, &vW));
    M2N_TRY(ctx->workspace("gep_U", sizeof(double) * (size_t)p * Np, &vU));
    M2N_TRY(ctx->workspace("gep_Y", sizeof(double) * (size_t)p * Np, &vY));
    size_t part_n = (size_t)gram_wg * p * p;
    if (part_n < (size_t)row_wg * 2 * K) part_n = (size_t)row_wg * 2 * K;
    M2N_TRY(ctx->workspace("gep_part", sizeof(double) * part_n, &vpart));
    M2N_TRY(ctx->workspace("gep_res", sizeof(double) * (size_t)row_wg * K, &vres));
    M2N_TRY(ctx->workspace("gep_Q", sizeof(double) * MAXP * MAXP, &vQ));
    M2N_TRY(ctx->workspace("gep_th", sizeof(double) * MAXP, &vth));
    M2N_TRY(ctx->workspace("gep_R", sizeof(double) * MAXP * MAXP, &vR));
    double *V = (double*)vV, *W = (double*)vW, *U = (double*)vU, *Y = (double*)vY;
    double *part = (double*)vpart, *res = (double*)vres, *Q = (double*)vQ, *th = (double*)vth,
           *Rm = (double*)vR;
    void* vt;
    M2N_TRY(ctx->workspace("gep_t", sizeof(double) * (size_t)N, &vt));
    M2N_HIP(hipMemcpyAsync(vt, t_dev, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, st));
    const double* td = (const double*)vt;

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
        void *vmap, *voff, *vH, *vc1, *vc2;
        const int pairs = (p + 1) / 2;
        M2N_TRY(ctx->workspace("gep_map", sizeof(int) * (size_t)M, &vmap));
        M2N_TRY(ctx->workspace("gep_off", sizeof(int) * (size_t)N, &voff));
        M2N_TRY(ctx->workspace("gep_H", sizeof(double) * (size_t)M, &vH));
        M2N_TRY(ctx->workspace("gep_c1", sizeof(cplx<double>) * (size_t)M * pairs, &vc1));
        M2N_TRY(ctx->workspace("gep_c2", sizeof(cplx<double>) * (size_t)M * pairs, &vc2));
        M2N_HIP(hipMemcpyAsync(voff, off.data(), sizeof(int) * (size_t)N, hipMemcpyHostToDevice, st));
        S.map = (int*)vmap;
        S.Hhat = (double*)vH;
        S.cbuf1 = (cplx<double>*)vc1;
        S.cbuf2 = (cplx<double>*)vc2;
        {
            M2N_PROF(ctx, st, "k_fill_int");
            hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, S.map, M, -1);
        }
        {
            M2N_PROF(ctx, st, "k_lattice_map");
            hipLaunchKernelGGL(k_lattice_map, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                               (const int*)voff, N, S.map);
        }
        // Hhat = FFT(h) / (M cB)
        {
            M2N_PROF(ctx, st, "k_toep_kernel");
            hipLaunchKernelGGL(k_toep_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                               S.cbuf2, M, Sspan, fw);
        }
        M2N_HIP(hipGetLastError());
        {
            ConvArgs a{};
            a.src = S.cbuf2;
            a.dst = S.cbuf1;
            void* vs;   // pass-A scratch, distinct from source and destination
            M2N_TRY(ctx->workspace("gep_hs", sizeof(cplx<double>) * (size_t)M, &vs));
            cplx<double>* scratch = (cplx<double>*)vs;
            M2N_TRY(run_fft64(S.fft, st, a, 1, SRC_DIRECT, DST_DIRECT, scratch));
        }
        {
            M2N_PROF(ctx, st, "k_real_scale");
            hipLaunchKernelGGL(k_real_scale, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                               (const cplx<double>*)S.cbuf1, M, 1.0 / ((double)M * cB), S.Hhat);
        }
        M2N_HIP(hipGetLastError());
        M2N_HIP(hipMemsetAsync(W, 0, sizeof(double) * (size_t)p * Np, st));
        scale = std::sqrt(2.0 * fw / cB);
        int status = 0;
        // the solve below must finish while the FFT plan is alive
        {
            // ---- subspace iteration
            dim3 g2((unsigned)((Np + 255) / 256), (unsigned)p);
            {
                M2N_PROF(ctx, st, "k_randinit");
                hipLaunchKernelGGL(k_randinit, g2, dim3(256), 0, st, U, Np, N, p, (uint64_t)0x5EED);
            }
            M2N_HIP(hipGetLastError());
            auto cholqr = [&](double* src, double* dst) -> int {
                {
                    M2N_PROF(ctx, st, "k_gram");
                    hipLaunchKernelGGL(k_gram, dim3(gram_wg), dim3(GNT), 0, st, src, src, Np, N, p, p, cpw,
                                       nchunks, part);
                }
                {
                    M2N_PROF(ctx, st, "k_chol_small");
                    hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(64), 0, st, part, gram_wg, p, Rm);
                }
                {
                    M2N_PROF(ctx, st, "k_trsm_rows");
                    hipLaunchKernelGGL(k_trsm_rows, dim3(row_wg), dim3(GNT), 0, st, src, Rm, Np, N, p, dst);
                }
                M2N_HIP(hipGetLastError());
                return M2N_OK;
            };
            M2N_TRY(cholqr(U, V));
            M2N_TRY(cholqr(V, V));
            std::vector<double> hres((size_t)row_wg * K);
            double prev = 1e300;
            bool ok = false;
            for (int it = 0; it < 40; ++it) {
                M2N_TRY(S.apply(V, W));
                {
                    M2N_PROF(ctx, st, "k_gram");
                    hipLaunchKernelGGL(k_gram, dim3(gram_wg), dim3(GNT), 0, st, V, W, Np, N, p, p, cpw,
                                       nchunks, part);
                }
                {
                    M2N_PROF(ctx, st, "k_rr");
                    hipLaunchKernelGGL(k_rr, dim3(1), dim3(64), 0, st, part, gram_wg, p, Q, th);
                }
                {
                    M2N_PROF(ctx, st, "k_rotate");
                    hipLaunchKernelGGL(k_rotate, dim3(row_wg), dim3(GNT), 0, st, V, W, Q, th, Np, N, p, K,
                                       Y, U, res);
                }
                M2N_HIP(hipGetLastError());
                M2N_HIP(hipMemcpyAsync(hres.data(), res, sizeof(double) * hres.size(),
                                       hipMemcpyDeviceToHost, st));
                M2N_HIP(hipStreamSynchronize(st));
                double rmax = 0.0;
                for (int k = 0; k < K; ++k) {
                    double s = 0.0;
                    for (int g = 0; g < row_wg; ++g) s += hres[(size_t)g * K + k];
                    rmax = std::fmax(rmax, std::sqrt(s));
                }
                if (p == N || rmax <= 1e-13 || (it >= 3 && rmax > 0.5 * prev && rmax <= 1e-10)) {
                    ok = true;
                    break;
                }
                prev = rmax;
                M2N_TRY(cholqr(U, V));
                M2N_TRY(cholqr(V, V));
            }
            if (!ok) status = M2N_ERR_NO_CONVERGE;
        }
        if (status != M2N_OK) {
            set_error("subspace iteration did not converge");
            return status;
        }
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
        dim3 gs((unsigned)((Np + 255) / 256), (unsigned)Np);
        {
            M2N_PROF(ctx, st, "k_gen_sinc");
            hipLaunchKernelGGL(k_gen_sinc, gs, dim3(256), 0, st, td, N, Np, fmax, 1.0, S.RB);
        }
        {
            M2N_PROF(ctx, st, "k_gen_sinc");
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
                {
                    M2N_PROF(ctx, st, "k_syrk");
                    hipLaunchKernelGGL(k_syrk, dim3(ntiles), dim3(GNT), 0, st, S.RB, Np, kb, S.nblk, S.nz);
                }
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
        dim3 g2((unsigned)((Np + 255) / 256), (unsigned)p);
        {
            M2N_PROF(ctx, st, "k_randinit");
            hipLaunchKernelGGL(k_randinit, g2, dim3(256), 0, st, U, Np, N, p, (uint64_t)0x5EED);
        }
        M2N_HIP(hipGetLastError());
        auto cholqr = [&](double* src, double* dst) -> int {
            {
                M2N_PROF(ctx, st, "k_gram");
                hipLaunchKernelGGL(k_gram, dim3(gram_wg), dim3(GNT), 0, st, src, src, Np, N, p, p, cpw,
                                   nchunks, part);
            }
            {
                M2N_PROF(ctx, st, "k_chol_small");
                hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(64), 0, st, part, gram_wg, p, Rm);
            }
            {
                M2N_PROF(ctx, st, "k_trsm_rows");
                hipLaunchKernelGGL(k_trsm_rows, dim3(row_wg), dim3(GNT), 0, st, src, Rm, Np, N, p, dst);
            }
            M2N_HIP(hipGetLastError());
            return M2N_OK;
        };
        M2N_TRY(cholqr(U, V));
        M2N_TRY(cholqr(V, V));
        std::vector<double> hres((size_t)row_wg * K);
        double prev = 1e300;
        bool ok = false;
        for (int it = 0; it < 40; ++it) {
            M2N_TRY(S.apply(V, W));
            {
                M2N_PROF(ctx, st, "k_gram");
                hipLaunchKernelGGL(k_gram, dim3(gram_wg), dim3(GNT), 0, st, V, W, Np, N, p, p, cpw, nchunks,
                                   part);
            }
            {
                M2N_PROF(ctx, st, "k_rr");
                hipLaunchKernelGGL(k_rr, dim3(1), dim3(64), 0, st, part, gram_wg, p, Q, th);
            }
            {
                M2N_PROF(ctx, st, "k_rotate");
                hipLaunchKernelGGL(k_rotate, dim3(row_wg), dim3(GNT), 0, st, V, W, Q, th, Np, N, p, K, Y, U,
                                   res);
            }
            M2N_HIP(hipGetLastError());
            M2N_HIP(hipMemcpyAsync(hres.data(), res, sizeof(double) * hres.size(),
                                   hipMemcpyDeviceToHost, st));
            M2N_HIP(hipStreamSynchronize(st));
            double rmax = 0.0;
            for (int k = 0; k < K; ++k) {
                double s = 0.0;
                for (int g = 0; g < row_wg; ++g) s += hres[(size_t)g * K + k];
                rmax = std::fmax(rmax, std::sqrt(s));
            }
            if (p == N || rmax <= 1e-13 || (it >= 3 && rmax > 0.5 * prev && rmax <= 1e-10)) {
                ok = true;
                break;
            }
            prev = rmax;
            M2N_TRY(cholqr(U, V));
            M2N_TRY(cholqr(V, V));
        }
        if (!ok) {
            set_error("subspace iteration did not converge");
            return M2N_ERR_NO_CONVERGE;
        }
        // y -> L^{-T} y for the first K Ritz vectors (solve on all p columns)
        const int psave = S.p;
        M2N_TRY(S.trsv(Y, 1));
        S.p = psave;
    }
    // ---- sign convention, scale, output
    {
        M2N_PROF(ctx, st, "k_sign_sums");
        hipLaunchKernelGGL(k_sign_sums, dim3(row_wg), dim3(GNT), 0, st, Y, Np, N, K, td, part);
    }
    const int fin_wg = (int)((N + GNT - 1) / GNT);
    {
        M2N_PROF(ctx, st, "k_finalize");
        hipLaunchKernelGGL(k_finalize, dim3(fin_wg), dim3(GNT), 0, st, Y, Np, N, K, scale, part,
                           row_wg, th, w_out, lambda_out);
    }
    M2N_HIP(hipGetLastError());
    M2N_HIP(hipStreamSynchronize(st));
    return M2N_OK;
}

}  // namespace m2n
