// Type-1 NuFFT of the K tapered sequences onto the I band centres, fused with
// the multitaper average and the suboptimality estimate.
//
//   J_k(i) = sum_n w_k(t_n) x_n exp(-j 2 pi (f_lo + i df) t_n)     (Sec. 3.2)
//   P_i    = sum_k d_k |J_k(i)|^2, d_k = 1/K by default           (Sec. 3.2)
//   Ehat_i = (1/K) sum_k |lambda_k - 2 f_w lambda_k / D_k(i)|      (App. B)
//
// Band i is mode i' = i - h of the periodic coordinate theta_n = 2 pi frac(df t_n)
// (h = floor(I/2)), after the per-point pre-phase exp(-j 2 pi (f_lo + h df) t_n):
//   J_k(i) = sum_n c_{n,k} exp(-j i' theta_n),  c_{n,k} = w_k(t_n) x_n e^{...}.
// The sum is evaluated by spreading c onto an oversampled grid of nf >= 2 I
// cells with the exponential-of-semicircle kernel
//   phi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| <= 1, over w cells,
// a length-nf FFT, and division by the kernel's Fourier transform phihat(i').
//
// Grid layout for nf = N1 * N2 (two passes): cell l = l2 + N2 l1.
//   pass 1: a workgroup owns B consecutive columns l2 of one taper, spreads the
//           points that reach them into an LDS tile, runs the N1-point column
//           FFTs, multiplies by exp(-2 pi i l2 m1 / nf) and writes G[k][m1][l2].
//   pass 2: a workgroup owns M consecutive rows m1, loops over the tapers,
//           runs the N2-point row FFTs (mode m = m1 + N1 m2), deconvolves,
//           keeps the I wanted modes and accumulates P (and J, E) in registers.
// Points are binned by the column block of their first cell (counting sort:
// per-workgroup histograms, one scan, scatter) so pass 1 reads contiguous runs.
// Small grids (nf <= 8192 FP32 / 4096 FP64) run the whole transform in one
// workgroup's LDS.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "fft_lds.hpp"
#include "m2n_common.hpp"

namespace m2n {

namespace {

constexpr int NT = 256;            // threads per workgroup, all NuFFT kernels
constexpr int PTS_PER_WG = 1024;   // points per workgroup in the binning kernels
constexpr int MAX_BINS = 1024;

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ void two_prod(double a, double b, double& hi, double& lo) {
    hi = a * b;
    lo = fma(a, b, -hi);
}

// (hi + lo) mod 1 in [0, 1)
__device__ __forceinline__ double frac01(double hi, double lo) {
    double r = (hi - floor(hi)) + lo;
    if (r < 0.0) r += 1.0;
    if (r >= 1.0) r -= 1.0;
    return r;
}

struct Geo {
    int l0;        // first cell of the kernel support, wrapped into [0, nf)
    double del;    // (unwrapped first cell) - u, in [-w/2, -w/2 + 1)
    double cre, cim;   // x_n exp(-j 2 pi (f_lo + h df) t_n)
    bool ok;
    bool integral;     // t_n is an integer
};

// Grid coordinate and pre-phase of one sample.  All in FP64; the products are
// split into exact hi + lo parts before reduction modulo 1.
__device__ __forceinline__ Geo point_geo(double t, double x, double f_lo, double df,
                                         int64_t h, int nf, int w) {
    Geo g;
    g.integral = (t == rint(t)) && fabs(t) < 4.0e15;
    if (!isfinite(t) || !isfinite(x)) {
        g.ok = false;
        g.l0 = 0;
        g.del = -0.5 * w;
        g.cre = g.cim = 0.0;
        return g;
    }
    double dh, dl;
    two_prod(df, t, dh, dl);
    const double u = (double)nf * frac01(dh, dl);    // nf is a power of two: exact
    if (!(u >= 0.0 && u < (double)nf)) {             // df * t overflowed
        g.ok = false;
        g.l0 = 0;
        g.del = -0.5 * w;
        g.cre = g.cim = 0.0;
        return g;
    }
    const double l0d = ceil(u - 0.5 * (double)w);
    int l0 = (int)l0d;
    g.del = l0d - u;
    if (l0 < 0) l0 += nf;
    g.l0 = l0;
    double ah, al, bh, bl;
    two_prod(f_lo, t, ah, al);
    const double hd = (double)h;
    two_prod(hd, dh, bh, bl);
    bl += hd * dl;
    const double ph = (ah - rint(ah)) + (bh - rint(bh)) + (al + bl);
    double s, c;
    sincospi(2.0 * ph, &s, &c);
    g.cre = x * c;
    g.cim = -x * s;
    g.ok = true;
    return g;
}

template <typename R>
__device__ __forceinline__ R es_kernel(R z, R beta) {
    R a = (R)1 - z * z;
    a = a > (R)0 ? a : (R)0;
    return exp(beta * (sqrt(a) - (R)1));
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block-wide sum for NT threads; every thread gets the result
__device__ __forceinline__ double block_sum(double v, double* scratch /* >= NT/64 */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += scratch[i];
    return s;
}

// ------------------------------------------------- binning (counting sort)
// K1a: per-workgroup bin histograms and lattice / finiteness flags.
__global__ __launch_bounds__(NT) void k_hist(const double* __restrict__ t,
                                             const double* __restrict__ x, int64_t N,
                                             double f_lo, double df, int64_t h, int nf,
                                             int w, int N2, int B, int nbins, int ppw,
                                             int* __restrict__ hist, int* __restrict__ flags) {
    __shared__ int sh[MAX_BINS];
    __shared__ int s_int, s_bad;
    const int wg = blockIdx.x;
    for (int b = threadIdx.x; b < nbins; b += NT) sh[b] = 0;
    if (threadIdx.x == 0) {
        s_int = 1;
        s_bad = 0;
    }
    __syncthreads();
    const int64_t n0 = (int64_t)wg * ppw;
    int my_int = 1, my_bad = 0;
    for (int j = threadIdx.x; j < ppw; j += NT) {
        const int64_t n = n0 + j;
        if (n >= N) break;
        Geo g = point_geo(t[n], x[n], f_lo, df, h, nf, w);
        my_int &= g.integral ? 1 : 0;
        my_bad |= g.ok ? 0 : 1;
        const int bin = (g.l0 & (N2 - 1)) / B;
        atomicAdd(&sh[bin], 1);
    }
    if (!my_int) atomicAnd(&s_int, 0);
    if (my_bad) atomicOr(&s_bad, 1);
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += NT) hist[(int64_t)wg * nbins + b] = sh[b];
    if (threadIdx.x == 0) flags[wg] = (s_int ? 1 : 0) | (s_bad ? 2 : 0);
}

// K1b: one workgroup.  off[wg][b] = start of (wg, b) in bin-major order,
// bin_off[b] = start of bin b.  Reduces the flags: diag[0] = 1 when R(B) is
// 2 f_max I (every t integer and 2 f_max a positive integer).  Clears the
// taper norms that pass 1 accumulates for Ehat.
constexpr int SCAN_LDS = 12288;   // (workgroup, bin) counts staged in LDS
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ hist, int nwg, int nbins,
                                               int* __restrict__ off, int* __restrict__ bin_off,
                                               const int* __restrict__ flags,
                                               unsigned* __restrict__ dev_err, int needE,
                                               double fmax, int* __restrict__ diag,
                                               double* __restrict__ norms, int K) {
    __shared__ int cnt[SCAN_LDS];
    __shared__ int tot[MAX_BINS + 1];
    __shared__ int s_int, s_bad;
    const int tid = threadIdx.x;
    const bool staged = (int64_t)nwg * nbins <= SCAN_LDS;
    if (tid == 0) {
        s_int = 1;
        s_bad = 0;
    }
    if (staged)
        for (int e = tid; e < nwg * nbins; e += blockDim.x) cnt[e] = hist[e];
    for (int k = tid; k < K; k += blockDim.x) norms[k] = 0.0;
    __syncthreads();
    for (int b = tid; b < nbins; b += blockDim.x) {
        int s = 0;
        for (int g = 0; g < nwg; ++g) s += staged ? cnt[g * nbins + b] : hist[(int64_t)g * nbins + b];
        tot[b] = s;
    }
    int li = 1, lb = 0;
    for (int g = tid; g < nwg; g += blockDim.x) {
        li &= flags[g] & 1;
        lb |= (flags[g] >> 1) & 1;
    }
    if (!li) atomicAnd(&s_int, 0);
    if (lb) atomicOr(&s_bad, 1);
    __syncthreads();
    // exclusive scan over the bins (one wavefront, 64-wide chunks)
    if (tid < 64) {
        int carry = 0;
        for (int c0 = 0; c0 < nbins; c0 += 64) {
            const int b = c0 + tid;
            int v = b < nbins ? tot[b] : 0;
            int incl = v;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(incl, o, 64);
                if (tid >= o) incl += u;
            }
            if (b < nbins) tot[b] = carry + incl - v;
            carry += __shfl(incl, 63, 64);
        }
        if (tid == 0) tot[nbins] = carry;
    }
    __syncthreads();
    for (int b = tid; b <= nbins; b += blockDim.x) bin_off[b] = tot[b];
    for (int b = tid; b < nbins; b += blockDim.x) {
        int run = tot[b];
        for (int g = 0; g < nwg; ++g) {
            const int c = staged ? cnt[g * nbins + b] : hist[(int64_t)g * nbins + b];
            if (staged) cnt[g * nbins + b] = run;
            else off[(int64_t)g * nbins + b] = run;
            run += c;
        }
    }
    __syncthreads();
    if (staged)
        for (int e = tid; e < nwg * nbins; e += blockDim.x) off[e] = cnt[e];
    if (tid == 0) {
        const double c = 2.0 * fmax;
        const int d = (s_int && c == rint(c) && c >= 1.0) ? 1 : 0;
        diag[0] = d;
        if (s_bad) atomicOr(dev_err, (unsigned)DEVERR_NONFINITE);
        if (needE && !d) atomicOr(dev_err, (unsigned)DEVERR_E_UNSUPPORTED);
    }
}

// K1c: scatter the points into bin order.
template <typename R>
__global__ __launch_bounds__(NT) void k_scatter(const double* __restrict__ t,
                                                const double* __restrict__ x, int64_t N,
                                                double f_lo, double df, int64_t h, int nf, int w,
                                                int N2, int B, int nbins, int ppw,
                                                const int* __restrict__ off,
                                                int* __restrict__ l0s, R* __restrict__ dels,
                                                cplx<R>* __restrict__ c0s,
                                                int* __restrict__ idxs) {
    __shared__ int cur[MAX_BINS];
    const int wg = blockIdx.x;
    for (int b = threadIdx.x; b < nbins; b += NT) cur[b] = 0;
    __syncthreads();
    const int64_t n0 = (int64_t)wg * ppw;
    for (int j = threadIdx.x; j < ppw; j += NT) {
        const int64_t n = n0 + j;
        if (n >= N) break;
        Geo g = point_geo(t[n], x[n], f_lo, df, h, nf, w);
        const int bin = (g.l0 & (N2 - 1)) / B;
        const int pos = off[(int64_t)wg * nbins + bin] + atomicAdd(&cur[bin], 1);
        l0s[pos] = g.l0;
        dels[pos] = (R)g.del;
        c0s[pos] = {(R)g.cre, (R)g.cim};
        idxs[pos] = (int)n;
    }
}

// -------------------------------------------------------------- pass 1
constexpr int NT1 = 512;   // threads per pass-1 workgroup
constexpr int NT2 = 512;   // threads per pass-2 workgroup

template <typename R, int N1, int B>
__global__ __launch_bounds__(NT1) void k_pass1(const int* __restrict__ l0s, const R* __restrict__ dels,
                                               const cplx<R>* __restrict__ c0s,
                                               const int* __restrict__ idxs,
                                               const int* __restrict__ bin_off,
                                               const double* __restrict__ wt, int64_t N,
                                               int log_N2, int nf, int w, R beta, int lookback,
                                               const cplx<R>* __restrict__ tw_g, int tws,
                                               const cplx<R>* __restrict__ tw_lo,
                                               const cplx<R>* __restrict__ tw_hi, int lo_bits,
                                               cplx<R>* __restrict__ inter, int needE,
                                               double* __restrict__ norms) {
    constexpr int LD = N1 + 1;
    __shared__ cplx<R> tile[B * LD];
    __shared__ cplx<R> tw[N1];
    __shared__ double nred;
    const int N2 = 1 << log_N2;
    const int nblk = N2 / B;
    const int blk = blockIdx.x % nblk;
    const int k = blockIdx.x / nblk;
    const int a = blk * B;
    for (int e = threadIdx.x; e < B * LD; e += NT1) tile[e] = {(R)0, (R)0};
    for (int j = threadIdx.x; j < N1; j += NT1) tw[j] = tw_g[j * tws];
    if (threadIdx.x == 0) nred = 0.0;
    __syncthreads();
    const R two_over_w = (R)2 / (R)w;
    const double* wk = wt + (int64_t)k * N;
    double nrm = 0.0;   // sum of w_k^2 over this block's own points (for Ehat)
    for (int q = 0; q <= lookback; ++q) {
        int bb = blk - q;
        if (bb < 0) bb += nblk;
        const int s = bin_off[bb], e = bin_off[bb + 1];
        for (int j = s + threadIdx.x; j < e; j += NT1) {
            const int l0 = l0s[j];
            const R del = dels[j];
            const double wd = wk[idxs[j]];
            if (q == 0) nrm += wd * wd;
            const R wv = (R)wd;
            const cplx<R> c = cscale(c0s[j], wv);
            for (int r = 0; r < w; ++r) {
                int cell = l0 + r;
                if (cell >= nf) cell -= nf;
                const int cb = (cell & (N2 - 1)) - a;
                if (cb >= 0 && cb < B) {
                    const int row = cell >> log_N2;
                    const R phi = es_kernel<R>(((R)r + del) * two_over_w, beta);
                    atomicAdd(&tile[cb * LD + row].x, c.x * phi);
                    atomicAdd(&tile[cb * LD + row].y, c.y * phi);
                }
            }
        }
    }
    if (needE) {
        for (int o = 32; o > 0; o >>= 1) nrm += __shfl_xor(nrm, o, 64);
        if ((threadIdx.x & 63) == 0) atomicAdd(&nred, nrm);
    }
    __syncthreads();
    if (needE && threadIdx.x == 0) atomicAdd(&norms[k], nred);
    fft_lds<R, N1, B, NT1, LD>(tile, tw, 1);
    const int lo_mask = (1 << lo_bits) - 1;
    cplx<R>* out = inter + (int64_t)k * nf;
    for (int e = threadIdx.x; e < B * N1; e += NT1) {
        const int cb = e % B, m1 = e / B;
        const int q = (a + cb) * m1;    // < nf
        const cplx<R> twv = cmul(tw_lo[q & lo_mask], tw_hi[q >> lo_bits]);
        out[(int64_t)m1 * N2 + a + cb] = cmul(tile[cb * LD + m1], twv);
    }
}

// -------------------------------------------------------------- pass 2
// A workgroup owns M consecutive rows m1 and transforms KC tapers at a time
// (KC * M rows in LDS); every output mode is owned by one thread, which
// accumulates sum_k d_k |J_k|^2 across the tapers in a register.
template <typename R, int N2, int M, int KC>
__global__ __launch_bounds__(NT2) void k_pass2(const cplx<R>* __restrict__ inter, int K, int N1,
                                               int nf, int64_t I, int64_t h,
                                               const cplx<R>* __restrict__ tw_g, int tws,
                                               const R* __restrict__ inv_phihat,
                                               const double* __restrict__ dk,
                                               R* __restrict__ P, R* __restrict__ E,
                                               const double* __restrict__ norms,
                                               const int* __restrict__ diag,
                                               const double* __restrict__ lambda, double fmax,
                                               double fw, cplx<R>* __restrict__ J) {
    constexpr int LD = N2 + 1;
    constexpr int ROWS = KC * M;
    constexpr int OUT_IT = (M * (N2 / 2 + 2) + NT2 - 1) / NT2;
    __shared__ cplx<R> rows[ROWS * LD];
    __shared__ cplx<R> tw[N2];
    __shared__ R s_eval;
    const int m1_0 = blockIdx.x * M;
    for (int j = threadIdx.x; j < N2; j += NT2) tw[j] = tw_g[j * tws];
    if (E && threadIdx.x == 0) {
        // D_k = 2 f_max |w_k|^2 when R(B) = 2 f_max I
        double e = 0.0;
        const double c = 2.0 * fmax;
        for (int k = 0; k < K; ++k) e += fabs(lambda[k] - 2.0 * fw * lambda[k] / (c * norms[k]));
        s_eval = diag[0] ? (R)(e / (double)K) : (R)NAN;
    }
    // modes kept: m2 in [0, npos) (i' >= 0) and [m2neg0, N2) (i' < 0)
    int npos = (int)((I - h + N1 - 1) / N1);
    if (npos > N2) npos = N2;
    int m2neg0 = (int)((nf - h) / N1);
    if (m2neg0 < npos) m2neg0 = npos;
    const int nneg = N2 - m2neg0;
    int nout = M * (npos + nneg);
    if (nout > OUT_IT * NT2) nout = OUT_IT * NT2;   // cannot happen for nf >= 2 I
    R acc[OUT_IT];
#pragma unroll
    for (int it = 0; it < OUT_IT; ++it) acc[it] = (R)0;
    for (int kc0 = 0; kc0 < K; kc0 += KC) {
        const int nk = K - kc0 < KC ? K - kc0 : KC;
        for (int e = threadIdx.x; e < ROWS * N2; e += NT2) {
            const int r = e / N2, l2 = e - r * N2;
            const int kq = r / M, mm = r - kq * M;
            cplx<R> v = {(R)0, (R)0};
            if (kq < nk)
                v = inter[(int64_t)(kc0 + kq) * nf + (int64_t)(m1_0 + mm) * N2 + l2];
            rows[r * LD + l2] = v;
        }
        __syncthreads();
        fft_lds<R, N2, ROWS, NT2, LD>(rows, tw, 1);
#pragma unroll
        for (int it = 0; it < OUT_IT; ++it) {
            const int e = threadIdx.x + it * NT2;
            if (e < nout) {
                const int mm = e % M, c = e / M;
                const int m2 = c < npos ? c : m2neg0 + (c - npos);
                const int64_t m = (int64_t)(m1_0 + mm) + (int64_t)N1 * m2;
                const int64_t kk = m < nf / 2 ? m : m - nf;
                const int64_t i = kk + h;
                if (i >= 0 && i < I) {
                    const R s = inv_phihat[kk < 0 ? -kk : kk];
                    for (int kq = 0; kq < nk; ++kq) {
                        const cplx<R> v = cscale(rows[(kq * M + mm) * LD + m2], s);
                        const R d = dk ? (R)dk[kc0 + kq] : (R)1 / (R)K;
                        acc[it] += d * (v.x * v.x + v.y * v.y);
                        if (J) J[(int64_t)(kc0 + kq) * I + i] = v;
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < OUT_IT; ++it) {
        const int e = threadIdx.x + it * NT2;
        if (e < nout) {
            const int mm = e % M, c = e / M;
            const int m2 = c < npos ? c : m2neg0 + (c - npos);
            const int64_t m = (int64_t)(m1_0 + mm) + (int64_t)N1 * m2;
            const int64_t kk = m < nf / 2 ? m : m - nf;
            const int64_t i = kk + h;
            if (i >= 0 && i < I) {
                if (P) P[i] = acc[it];
                if (E) E[i] = s_eval;
            }
        }
    }
}

// ------------------------------------------------- single-workgroup path
template <typename R, int NF>
__global__ __launch_bounds__(NT) void k_small(const double* __restrict__ t,
                                              const double* __restrict__ x, int64_t N,
                                              const double* __restrict__ wt, int K, double f_lo,
                                              double df, int64_t I, int64_t h, int w, R beta,
                                              const cplx<R>* __restrict__ tw, int tws,
                                              const R* __restrict__ inv_phihat,
                                              const double* __restrict__ dk,
                                              const double* __restrict__ lambda, double fmax,
                                              double fw, unsigned* __restrict__ dev_err,
                                              R* __restrict__ P, R* __restrict__ E,
                                              cplx<R>* __restrict__ J) {
    constexpr int OUT_IT = (NF / 2 + NT - 1) / NT;
    __shared__ cplx<R> grid[NF];
    __shared__ double red[NT / 64];
    __shared__ int s_int, s_bad;
    if (threadIdx.x == 0) {
        s_int = 1;
        s_bad = 0;
    }
    R acc[OUT_IT];
#pragma unroll
    for (int it = 0; it < OUT_IT; ++it) acc[it] = (R)0;
    const R two_over_w = (R)2 / (R)w;
    double esum = 0.0;
    for (int k = 0; k < K; ++k) {
        for (int e = threadIdx.x; e < NF; e += NT) grid[e] = {(R)0, (R)0};
        __syncthreads();
        const double* wk = wt + (int64_t)k * N;
        double nrm = 0.0;
        int my_int = 1, my_bad = 0;
        for (int64_t n = threadIdx.x; n < N; n += NT) {
            const Geo g = point_geo(t[n], x[n], f_lo, df, h, NF, w);
            my_int &= g.integral ? 1 : 0;
            my_bad |= g.ok ? 0 : 1;
            const double wv = wk[n];
            nrm += wv * wv;
            const cplx<R> c = {(R)(g.cre * wv), (R)(g.cim * wv)};
            const R del = (R)g.del;
            for (int r = 0; r < w; ++r) {
                int cell = g.l0 + r;
                if (cell >= NF) cell -= NF;
                const R phi = es_kernel<R>(((R)r + del) * two_over_w, beta);
                atomicAdd(&grid[cell].x, c.x * phi);
                atomicAdd(&grid[cell].y, c.y * phi);
            }
        }
        if (!my_int) atomicAnd(&s_int, 0);
        if (my_bad) atomicOr(&s_bad, 1);
        nrm = block_sum(nrm, red);   // contains barriers
        if (E && lambda) {
            const double c = 2.0 * fmax;
            esum += fabs(lambda[k] - 2.0 * fw * lambda[k] / (c * nrm));
        }
        fft_lds<R, NF, 1, NT, NF>(grid, tw, tws);
        const R d = dk ? (R)dk[k] : (R)1 / (R)K;
#pragma unroll
        for (int it = 0; it < OUT_IT; ++it) {
            const int64_t i = threadIdx.x + (int64_t)it * NT;
            if (i < I) {
                const int64_t kk = i - h;
                const int64_t m = kk < 0 ? kk + NF : kk;
                const R s = inv_phihat[kk < 0 ? -kk : kk];
                const cplx<R> v = cscale(grid[m], s);
                acc[it] += d * (v.x * v.x + v.y * v.y);
                if (J) J[(int64_t)k * I + i] = v;
            }
        }
        __syncthreads();
    }
    const double c = 2.0 * fmax;
    const bool diag = s_int && c == rint(c) && c >= 1.0;
    const R ev = diag ? (R)(esum / (double)K) : (R)NAN;
    if (threadIdx.x == 0) {
        if (s_bad) atomicOr(dev_err, (unsigned)DEVERR_NONFINITE);
        if (E && !diag) atomicOr(dev_err, (unsigned)DEVERR_E_UNSUPPORTED);
    }
#pragma unroll
    for (int it = 0; it < OUT_IT; ++it) {
        const int64_t i = threadIdx.x + (int64_t)it * NT;
        if (i < I) {
            if (P) P[i] = acc[it];
            if (E) E[i] = ev;
        }
    }
}

// deconvolution table 1/phihat(k), k = 0..kmax, by Gauss-Legendre quadrature
//   phihat(k) = (w/2) int_{-1}^{1} phi(z) cos(pi k w z / nf) dz
template <typename R>
__global__ void k_phihat(int64_t kmax, int nf, int w, double beta, const double* __restrict__ gx,
                         const double* __restrict__ gw, int ng, R* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kmax) return;
    double s = 0.0;
    for (int q = 0; q < ng; ++q) {
        const double z = gx[q];
        const double phi = exp(beta * (sqrt(fmax(1.0 - z * z, 0.0)) - 1.0));
        s += gw[q] * phi * cospi((double)k * (double)w * z / (double)nf);
    }
    out[k] = (R)(1.0 / (0.5 * (double)w * s));
}

// ------------------------------------------------------------ host helpers
template <typename R>
std::vector<cplx<R>> twiddles(int64_t n, int64_t count, int64_t stride) {
    // exp(-2 pi i j stride / n) for j < count
    std::vector<cplx<R>> v(count);
    for (int64_t j = 0; j < count; ++j) {
        const long double a = -2.0L * (long double)M_PI * (long double)((j * stride) % n) / (long double)n;
        v[j] = {(R)std::cos((double)a), (R)std::sin((double)a)};
    }
    return v;
}

int ilog2i(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

template <typename R>
int upload(Ctx* ctx, DevBuf& b, const std::vector<R>& v) {
    M2N_TRY(ctx->alloc(b, v.size() * sizeof(R)));
    M2N_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(R), hipMemcpyHostToDevice));
    return M2N_OK;
}

template <typename R>
int build_plan(Ctx* ctx, NufftPlan& p) {
    const int cs = (int)sizeof(cplx<R>);
    const int single_max = sizeof(R) == 4 ? 8192 : 4096;
    p.single = p.nf <= single_max;
    int Nt;
    if (p.single) {
        Nt = p.nf;
    } else {
        int L = p.log_nf;
        int l1 = L / 2;
        if (l1 > 10) l1 = 10;
        p.N1 = 1 << l1;
        p.N2 = p.nf / p.N1;
        if (p.N2 > 4096) {
            set_error("band count too large for this build (nf = %d)", p.nf);
            return M2N_ERR_UNSUPPORTED;
        }
        p.B = 65536 / (p.N1 * cs);
        if (p.B > 32) p.B = 32;
        if (p.B > p.N2 / 2) p.B = p.N2 / 2;
        p.lookback = (p.w - 1 + p.B - 1) / p.B;
        if (p.lookback >= p.N2 / p.B || p.N2 / p.B > MAX_BINS) {
            set_error("unsupported grid split (N2 = %d, B = %d, w = %d)", p.N2, p.B, p.w);
            return M2N_ERR_UNSUPPORTED;
        }
        // pass 2: KC tapers x M rows of N2 (+1 pad) values plus the N2-entry
        // twiddle table must fit the 160 KB LDS of a compute unit
        int rows_max = 1;
        while (2 * rows_max * (p.N2 + 1) * cs + p.N2 * cs <= 160000) rows_max *= 2;
        p.KC = rows_max < 8 ? rows_max : 8;
        p.M = rows_max / p.KC;
        if (p.M > 4) p.M = 4;
        p.lo_bits = (p.log_nf + 1) / 2;
        Nt = p.N1 > p.N2 ? p.N1 : p.N2;
        M2N_TRY(upload(ctx, p.tw_lo, twiddles<R>(p.nf, int64_t(1) << p.lo_bits, 1)));
        M2N_TRY(upload(ctx, p.tw_hi, twiddles<R>(p.nf, p.nf >> p.lo_bits, int64_t(1) << p.lo_bits)));
    }
    p.tw_len = Nt;
    M2N_TRY(upload(ctx, p.tw_fft, twiddles<R>(Nt, Nt, 1)));
    // deconvolution table
    int64_t kmax = p.h > (p.I - 1 - p.h) ? p.h : (p.I - 1 - p.h);
    p.kmax = kmax;
    const int ng = 2 * (2 + (3 * p.w + 1) / 2) + 8;
    std::vector<double> gx, gw;
    gauss_legendre(ng, gx, gw);
    DevBuf dgx, dgw;
    M2N_TRY(upload(ctx, dgx, gx));
    M2N_TRY(upload(ctx, dgw, gw));
    M2N_TRY(ctx->alloc(p.inv_phihat, (size_t)(kmax + 1) * sizeof(R)));
    const int64_t nthr = kmax + 1;
    {
        hipLaunchKernelGGL(k_phihat<R>, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, 0, kmax,
                           p.nf, p.w, p.beta, (const double*)dgx.p, (const double*)dgw.p, ng,
                           (R*)p.inv_phihat.p);
    }
    M2N_HIP(hipGetLastError());
    M2N_HIP(hipDeviceSynchronize());
    ctx->release(dgx);
    ctx->release(dgw);
    return M2N_OK;
}

int get_plan(Ctx* ctx, int64_t I, int prec, double tol, NufftPlan** out) {
    if (tol <= 0.0) tol = (prec == M2N_FP32) ? 1e-6 : 1e-12;
    int w = (int)std::ceil(-std::log10(tol)) + 1;
    if (w < 4) w = 4;
    if (prec == M2N_FP32 && w > 8) w = 8;
    if (w > 16) w = 16;
    auto key = std::make_tuple(I, prec, w);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
        *out = it->second.get();
        return M2N_OK;
    }
    auto p = std::make_unique<NufftPlan>();
    p->I = I;
    p->h = I / 2;
    p->prec = prec;
    p->w = w;
    p->beta = 2.30 * w;
    int64_t nf = 64;
    while (nf < 2 * I) nf *= 2;
    while (nf < 4 * w) nf *= 2;
    p->nf = (int)nf;
    p->log_nf = ilog2i(nf);
    int st = prec == M2N_FP32 ? build_plan<float>(ctx, *p) : build_plan<double>(ctx, *p);
    if (st != M2N_OK) {
        ctx->release(p->tw_fft);
        ctx->release(p->tw_lo);
        ctx->release(p->tw_hi);
        ctx->release(p->inv_phihat);
        return st;
    }
    *out = p.get();
    ctx->plans.emplace(key, std::move(p));
    return M2N_OK;
}

// ---------------------------------------------------------- dispatchers
template <typename R>
void launch_small(const NufftPlan& p, hipStream_t st, const double* t, const double* x,
                  int64_t N, const double* w, int K, double f_lo, double df,
                  const double* dk, const double* lambda, double fmax, double fw,
                  unsigned* dev_err, R* P, R* E, cplx<R>* J) {
#define M2N_SMALL(NFV)                                                                         \
    case NFV:                                                                                  \
        hipLaunchKernelGGL((k_small<R, NFV>), dim3(1), dim3(NT), 0, st, t, x, N, w, K, f_lo,    \
                           df, p.I, p.h, p.w, (R)p.beta, (const cplx<R>*)p.tw_fft.p, 1,        \
                           (const R*)p.inv_phihat.p, dk, lambda, fmax, fw, dev_err, P, E, J); \
        break;
    switch (p.nf) {
        M2N_SMALL(64)
        M2N_SMALL(128)
        M2N_SMALL(256)
        M2N_SMALL(512)
        M2N_SMALL(1024)
        M2N_SMALL(2048)
        M2N_SMALL(4096)
        default:
            if constexpr (sizeof(R) == 4) {
                switch (p.nf) { M2N_SMALL(8192) default: break; }
            }
            break;
    }
#undef M2N_SMALL
}

template <typename R>
int launch_pass1(const NufftPlan& p, hipStream_t st, dim3 grid, const int* l0s, const R* dels,
                 const cplx<R>* c0s, const int* idxs, const int* bin_off, const double* w,
                 int64_t N, cplx<R>* inter, int needE, double* norms) {
    const int tws = p.tw_len / p.N1;
    const int logN2 = ilog2i(p.N2);
#define M2N_P1(N1V, BV)                                                                          \
    if (p.N1 == N1V && p.B == BV) {                                                              \
        hipLaunchKernelGGL((k_pass1<R, N1V, BV>), grid, dim3(NT1), 0, st, l0s, dels, c0s, idxs,  \
                           bin_off, w, N, logN2, p.nf, p.w, (R)p.beta, p.lookback,               \
                           (const cplx<R>*)p.tw_fft.p, tws, (const cplx<R>*)p.tw_lo.p,           \
                           (const cplx<R>*)p.tw_hi.p, p.lo_bits, inter, needE, norms);           \
        return M2N_OK;                                                                           \
    }
    if constexpr (sizeof(R) == 4) {
        M2N_P1(64, 32) M2N_P1(128, 32) M2N_P1(256, 32) M2N_P1(512, 16) M2N_P1(1024, 8)
    } else {
        M2N_P1(64, 32) M2N_P1(128, 32) M2N_P1(256, 16) M2N_P1(512, 8) M2N_P1(1024, 4)
    }
#undef M2N_P1
    set_error("no pass-1 kernel for N1 = %d, B = %d", p.N1, p.B);
    return M2N_ERR_UNSUPPORTED;
}

// rows-per-workgroup choice for pass 2: largest M the LDS budget allows that
// still gives at least two workgroups per compute unit
inline int pass2_rows(const NufftPlan& p, int cu_count) {
    int M = p.M;
    while (M > 1 && (p.N1 / M) < 2 * cu_count) M /= 2;
    return M;
}

template <typename R>
int launch_pass2(const NufftPlan& p, hipStream_t st, int M, const cplx<R>* inter, int K,
                 const double* dk, R* P, R* E, const double* norms, const int* diag,
                 const double* lambda, double fmax, double fw, cplx<R>* J) {
    const int tws = p.tw_len / p.N2;
    dim3 grid(p.N1 / M);
#define M2N_P2(N2V, MV, KCV)                                                                     \
    if (p.N2 == N2V && M == MV && p.KC == KCV) {                                                 \
        hipLaunchKernelGGL((k_pass2<R, N2V, MV, KCV>), grid, dim3(NT2), 0, st, inter, K, p.N1,   \
                           p.nf, p.I, p.h, (const cplx<R>*)p.tw_fft.p, tws,                      \
                           (const R*)p.inv_phihat.p, dk, P, E, norms, diag, lambda, fmax, fw,    \
                           J);                                                                   \
        return M2N_OK;                                                                           \
    }
    if constexpr (sizeof(R) == 4) {
        M2N_P2(128, 1, 8) M2N_P2(128, 2, 8) M2N_P2(128, 4, 8)
        M2N_P2(256, 1, 8) M2N_P2(256, 2, 8) M2N_P2(256, 4, 8)
        M2N_P2(512, 1, 8) M2N_P2(512, 2, 8) M2N_P2(512, 4, 8)
        M2N_P2(1024, 1, 8) M2N_P2(1024, 2, 8)
        M2N_P2(2048, 1, 8) M2N_P2(4096, 1, 2)
    } else {
        M2N_P2(128, 1, 8) M2N_P2(128, 2, 8) M2N_P2(128, 4, 8)
        M2N_P2(256, 1, 8) M2N_P2(256, 2, 8) M2N_P2(256, 4, 8)
        M2N_P2(512, 1, 8) M2N_P2(512, 2, 8)
        M2N_P2(1024, 1, 8) M2N_P2(2048, 1, 2) M2N_P2(4096, 1, 1)
    }
#undef M2N_P2
    set_error("no pass-2 kernel for N2 = %d, M = %d, KC = %d", p.N2, M, p.KC);
    return M2N_ERR_UNSUPPORTED;
}

template <typename R>
int run_typed(Ctx* ctx, hipStream_t st, const NufftPlan& p, const double* t, const double* x,
              int64_t N, const double* w, int K, double f_lo, double df, const double* dk,
              const double* lambda, double fmax, double fw, void* Pv, void* Ev, void* Jv) {
    R* P = (R*)Pv;
    R* E = (R*)Ev;
    cplx<R>* J = (cplx<R>*)Jv;
    if (p.single) {
        M2N_PROF(ctx, st, "k_small");
        launch_small<R>(p, st, t, x, N, w, K, f_lo, df, dk, lambda, fmax, fw, ctx->dev_err, P, E,
                        J);
        M2N_HIP(hipGetLastError());
        return M2N_OK;
    }
    const int nbins = p.N2 / p.B;
    // points per binning workgroup: at least PTS_PER_WG, and few enough
    // workgroups that the scan can stage every (workgroup, bin) count in LDS
    int64_t ppw = PTS_PER_WG;
    while ((N + ppw - 1) / ppw * nbins > SCAN_LDS && ppw < (int64_t(1) << 20)) ppw *= 2;
    const int64_t nwg64 = (N + ppw - 1) / ppw;
    if (nwg64 > (1 << 20)) {
        set_error("N too large");
        return M2N_ERR_ARG;
    }
    const int nwg = (int)nwg64;
    const bool needE = E != nullptr;
    void *hist, *off, *binoff, *flags, *l0s, *dels, *c0s, *idxs, *inter, *norms, *diag;
    M2N_TRY(ctx->workspace("nu_hist", sizeof(int) * (size_t)nwg * nbins, &hist));
    M2N_TRY(ctx->workspace("nu_off", sizeof(int) * (size_t)nwg * nbins, &off));
    M2N_TRY(ctx->workspace("nu_binoff", sizeof(int) * (size_t)(nbins + 1), &binoff));
    M2N_TRY(ctx->workspace("nu_flags", sizeof(int) * (size_t)nwg, &flags));
    M2N_TRY(ctx->workspace("nu_l0", sizeof(int) * (size_t)N, &l0s));
    M2N_TRY(ctx->workspace("nu_del", sizeof(R) * (size_t)N, &dels));
    M2N_TRY(ctx->workspace("nu_c0", sizeof(cplx<R>) * (size_t)N, &c0s));
    M2N_TRY(ctx->workspace("nu_idx", sizeof(int) * (size_t)N, &idxs));
    M2N_TRY(ctx->workspace("nu_inter", sizeof(cplx<R>) * (size_t)K * p.nf, &inter));
    M2N_TRY(ctx->workspace("nu_norms", sizeof(double) * 64, &norms));
    M2N_TRY(ctx->workspace("nu_diag", 64, &diag));
    {
        M2N_PROF(ctx, st, "k_hist");
        hipLaunchKernelGGL(k_hist, dim3(nwg), dim3(NT), 0, st, t, x, N, f_lo, df, p.h, p.nf, p.w,
                           p.N2, p.B, nbins, (int)ppw, (int*)hist, (int*)flags);
    }
    {
        M2N_PROF(ctx, st, "k_scan");
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, (const int*)hist, nwg, nbins,
                           (int*)off, (int*)binoff, (const int*)flags, ctx->dev_err, needE ? 1 : 0,
                           fmax, (int*)diag, (double*)norms, K);
    }
    {
        M2N_PROF(ctx, st, "k_scatter");
        hipLaunchKernelGGL(k_scatter<R>, dim3(nwg), dim3(NT), 0, st, t, x, N, f_lo, df, p.h, p.nf,
                           p.w, p.N2, p.B, nbins, (int)ppw, (const int*)off, (int*)l0s, (R*)dels,
                           (cplx<R>*)c0s, (int*)idxs);
    }
    M2N_HIP(hipGetLastError());
    {
        M2N_PROF(ctx, st, "k_pass1");
        M2N_TRY(launch_pass1<R>(p, st, dim3((unsigned)(K * nbins)), (const int*)l0s, (const R*)dels,
                                (const cplx<R>*)c0s, (const int*)idxs, (const int*)binoff, w, N,
                                (cplx<R>*)inter, needE ? 1 : 0, (double*)norms));
    }
    M2N_HIP(hipGetLastError());
    {
        M2N_PROF(ctx, st, "k_pass2");
        M2N_TRY(launch_pass2<R>(p, st, pass2_rows(p, ctx->cu_count), (const cplx<R>*)inter, K, dk,
                                P, E, (const double*)norms, (const int*)diag, lambda, fmax, fw, J));
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

}  // namespace

int nufft_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N,
              const double* w, int K, double f_lo, double df, int64_t I, int prec, double tol,
              const double* weights, const double* lambda, double fmax, double fw, void* P,
              void* E, void* J) {
    if (!t || !x || !w || N < 1 || K < 1 || K > 64 || I < 1 || I > (int64_t(1) << 21)) {
        set_error("bad argument (N = %lld, K = %d, I = %lld)", (long long)N, K, (long long)I);
        return M2N_ERR_ARG;
    }
    if (N > (int64_t(1) << 30)) {
        set_error("N too large");
        return M2N_ERR_ARG;
    }
    if (!std::isfinite(f_lo) || !std::isfinite(df) || !(df > 0.0)) {
        set_error("band grid must have finite f_lo and df > 0");
        return M2N_ERR_ARG;
    }
    if (prec != M2N_FP32 && prec != M2N_FP64) {
        set_error("prec must be M2N_FP32 or M2N_FP64");
        return M2N_ERR_ARG;
    }
    if (E && (!lambda || !(fmax > 0.0) || !(fw > 0.0))) {
        set_error("E needs lambda, fmax > 0 and fw > 0");
        return M2N_ERR_ARG;
    }
    NufftPlan* p = nullptr;
    M2N_TRY(get_plan(ctx, I, prec, tol, &p));
    if (prec == M2N_FP32)
        return run_typed<float>(ctx, st, *p, t, x, N, w, K, f_lo, df, weights, lambda, fmax, fw,
                                P, E, J);
    return run_typed<double>(ctx, st, *p, t, x, N, w, K, f_lo, df, weights, lambda, fmax, fw, P,
                             E, J);
}

}  // namespace m2n
