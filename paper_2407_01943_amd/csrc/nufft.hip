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
//   pass 1: a workgroup owns B consecutive columns l2 of one taper, gathers the
//           taper's values of the points that reach them by sample index,
//           spreads them into an LDS tile, runs the N1-point column FFTs,
//           multiplies by exp(-2 pi i l2 m1 / nf) and writes G[k][m1][l2].
//   pass 2: a workgroup owns M consecutive rows m1, loops over the tapers,
//           runs the N2-point row FFTs (mode m = m1 + N1 m2), deconvolves,
//           keeps the I wanted modes and accumulates P (and J, E) in registers;
//           for P and E alone on rows of 512, 1024 or 2048, one wavefront
//           transforms each taper's row by itself (k_pass2w).
// Points are binned by the column block of their first cell (counting sort:
// per-workgroup histograms, one scan, then the binned geometry with each
// point's sample index), so pass 1 reads contiguous runs.  The binning needs
// only t and x and can run before the tapers exist.
// Small grids (nf <= 8192 FP32 / 4096 FP64) run the whole transform in one
// workgroup's LDS.
//
// Every kernel serves one series or a batch: the per-series inputs, outputs
// and workspace are a NuSeries descriptor, passed by value for one series or
// as a device array indexed by blockIdx.y for a batch; NuArgs holds what the
// plan fixes (band count, grid split, tables).
#include <cmath>
#include <memory>
#include <cstdarg>
#include <cstring>

#include "fft_lds.hpp"
#include "m2n_common.hpp"

namespace m2n {

namespace {

constexpr int NT = 256;            // threads per workgroup, all NuFFT kernels
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

// FP32 spreading weights from the hardware square root and base-2
// exponential: phi <= 1 and the exponent error (a few ulps of |beta|) gives
// a relative error of about 1e-6 only where phi is already tiny
template <typename R>
__device__ __forceinline__ R es_spread(R z, R beta);
template <>
__device__ __forceinline__ float es_spread<float>(float z, float beta) {
    float a = 1.0f - z * z;
    a = a > 0.0f ? a : 0.0f;
    return __builtin_amdgcn_exp2f(beta * 1.4426950408889634f * (__builtin_amdgcn_sqrtf(a) - 1.0f));
}
template <>
__device__ __forceinline__ double es_spread<double>(double z, double beta) {
    return es_kernel<double>(z, beta);
}

// a pointer taken out of a descriptor, marked as global memory so that
// loads through it are global (not flat) loads
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gp(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

// inclusive scan over the 64 lanes with DPP: row shifts by 1, 2, 4 and 8
// within rows of 16, then each row total broadcast into the following rows
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// a double moved across lanes by a DPP pattern (both halves); lanes whose
// source is out of range or whose row is masked off receive 0
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_dbl(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over the 64 lanes in a fixed order (quad permutes, row shifts, row
// broadcasts); the total lands in lane 63
__device__ __forceinline__ double wave_sum_to63(double v) {
    v += dpp_dbl<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp_dbl<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp_dbl<0x114, 0xf>(v);   // row_shr:4
    v += dpp_dbl<0x118, 0xf>(v);   // row_shr:8
    v += dpp_dbl<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_dbl<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// Thomson F-statistic of one band from S_JW = sum_k J_k W_k(0), S_JJ =
// sum_k |J_k|^2 and S_WW = sum_k W_k(0)^2: with q = |S_JW|^2 / S_WW (the
// power of the fitted line C W(0)) the residual is S_JJ - q, and
// F = (K - 1) q / (S_JJ - q); +inf where the residual vanishes
template <typename R>
__device__ __forceinline__ R f_statistic(cplx<R> sjw, R sjj, R sww, int K) {
    const R q = (sjw.x * sjw.x + sjw.y * sjw.y) / sww;
    const R res = sjj - q;
    return res > (R)0 ? (R)(K - 1) * q / res : (R)INFINITY;
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

// ------------------------------------------------------ launch descriptors
struct NuSeries {
    const double* t;
    const double* x;
    const double* w;        // K x N tapers
    const double* lambda;   // for E
    const double* dk;       // weights or NULL
    void* P;
    void* E;
    void* J;
    void* F;       // Thomson F-statistic or NULL
    int* hist;     // [nwg][nbins] counts
    int* off;      // [nwg][nbins] scatter offsets
    int* binoff;   // [nbins + 1]
    int* flags;    // [nwg]
    int* l0s;      // [N] binned first cells
    void* dels;    // [N] R offsets
    double* cx;    // [N][2] pre-phased samples x_n e^{-j 2 pi (f_lo + h df) t_n}, bin order
    int* perm;     // [N] sample index n of each binned point
    void* inter;   // [K][nf] cplx<R> after pass 1
    double* nrm;   // [nbins][K] pass 1's per-block shares of sum_n w_k^2 (for E)
    double* wsp;   // [nbins][K] the same for sum_n w_k (for F)
    int* diag;     // [1] R(B) = 2 f_max I
    double* hrec;  // pinned host record of the t check, or NULL: [0] flags
                   // (bit 0 non-finite, bit 1 not increasing, bit 2 a t_n
                   // that is not an integer), [1] t_0, [2] t_{N-1}
    int64_t N;
    double f_lo, df, fmax, fw;
    int K, nwg, ppw, pad;
};

struct NuArgs {
    int64_t I, h;
    double beta;
    int nf, w, N1, N2, B, nbins, log_N2, lookback, tws1, tws2;
    const void* tw;          // FFT twiddles
    const void* inv_phihat;  // deconvolution table
    unsigned* dev_err;
};

// this workgroup's series
__device__ __forceinline__ NuSeries series_of(const NuSeries& d0, const NuSeries* D) {
    return D ? D[blockIdx.y] : d0;
}

// ------------------------------------------------- binning (counting sort)
// K1a: per-workgroup bin histograms and lattice / finiteness flags.
__global__ __launch_bounds__(NT) void k_hist(NuArgs a, NuSeries d0, const NuSeries* D) {
    const NuSeries d = series_of(d0, D);
    const int wg = blockIdx.x;
    if (wg >= d.nwg) return;
    __shared__ int sh[MAX_BINS];
    __shared__ int s_int, s_bad, s_ord;
    for (int b = threadIdx.x; b < a.nbins; b += NT) sh[b] = 0;
    if (threadIdx.x == 0) {
        s_int = 1;
        s_bad = 0;
        s_ord = 0;
    }
    __syncthreads();
    const int64_t n0 = (int64_t)wg * d.ppw;
    int my_int = 1, my_bad = 0, my_ord = 0;
    for (int j = threadIdx.x; j < d.ppw; j += NT) {
        const int64_t n = n0 + j;
        if (n >= d.N) break;
        const double tn = d.t[n];
        Geo g = point_geo(tn, d.x[n], d.f_lo, d.df, a.h, a.nf, a.w);
        my_int &= g.integral ? 1 : 0;
        my_bad |= g.ok ? 0 : 1;
        if (d.hrec && n > 0 && !(tn > d.t[n - 1])) my_ord = 1;
        const int bin = (g.l0 & (a.N2 - 1)) / a.B;
        atomicAdd(&sh[bin], 1);
    }
    if (!my_int) atomicAnd(&s_int, 0);
    if (my_bad) atomicOr(&s_bad, 1);
    if (my_ord) atomicOr(&s_ord, 1);
    __syncthreads();
    for (int b = threadIdx.x; b < a.nbins; b += NT) d.hist[(int64_t)wg * a.nbins + b] = sh[b];
    if (threadIdx.x == 0) d.flags[wg] = (s_int ? 1 : 0) | (s_bad ? 2 : 0) | (s_ord ? 4 : 0);
}

// the t check's record for the host (thread 0 of the series' last kernel
// that has seen every sample)
__device__ __forceinline__ void write_hrec(const NuSeries& d, bool integral, bool bad, bool ord) {
    if (!d.hrec) return;
    const int f = (bad ? 1 : 0) | (ord ? 2 : 0) | (integral ? 0 : 4);
    d.hrec[0] = (double)f;
    d.hrec[1] = d.t[0];
    d.hrec[2] = d.t[d.N - 1];
    __threadfence_system();
}

// K1b: one workgroup per series.  off[wg][b] = start of (wg, b) in bin-major
// order, binoff[b] = start of bin b.  Reduces the flags: diag[0] = 1 when
// R(B) is 2 f_max I (every t integer and 2 f_max a positive integer).
constexpr int SCAN_LDS = 12288;   // (workgroup, bin) counts staged in LDS
__global__ __launch_bounds__(1024) void k_scan(NuArgs a, NuSeries d0, const NuSeries* D) {
    const NuSeries d = series_of(d0, D);
    __shared__ int cnt[SCAN_LDS];
    __shared__ int tot[MAX_BINS + 1];
    __shared__ int s_int, s_bad, s_ord;
    const int tid = threadIdx.x;
    const int nwg = d.nwg, nbins = a.nbins;
    // staged: the counts held bin-major, cnt[b * nwgp + g], with an odd row
    // length so that both the wavefront reads along g and the strided
    // writes are free of bank conflicts
    const int nwgp = nwg | 1;
    const bool staged = (int64_t)nwgp * nbins <= SCAN_LDS;
    if (tid == 0) {
        s_int = 1;
        s_bad = 0;
        s_ord = 0;
    }
    if (staged) {
        // all of a thread's loads in flight at once (blockDim.x = 1024)
        constexpr int SU = SCAN_LDS / 1024;
        int v[SU];
#pragma unroll
        for (int i = 0; i < SU; ++i) {
            const int e = tid + i * 1024;
            v[i] = e < nwg * nbins ? d.hist[e] : 0;
        }
#pragma unroll
        for (int i = 0; i < SU; ++i) {
            const int e = tid + i * 1024;
            if (e < nwg * nbins) {
                const int g = e / nbins, b = e - g * nbins;
                cnt[b * nwgp + g] = v[i];
            }
        }
    }
    __syncthreads();
    if (staged) {
        // per bin, the exclusive scan along the workgroups (one wavefront per
        // bin, 64 workgroups per step); tot[b] = the bin's total
        const int lane = tid & 63, wv = tid >> 6, nw = (int)(blockDim.x >> 6);
        for (int b = wv; b < nbins; b += nw) {
            int carry = 0;
            for (int g0 = 0; g0 < nwg; g0 += 64) {
                const int g = g0 + lane;
                const int c = g < nwg ? cnt[b * nwgp + g] : 0;
                const int incl = wave_incl_scan(c);
                if (g < nwg) cnt[b * nwgp + g] = carry + incl - c;
                carry += __builtin_amdgcn_readlane(incl, 63);
            }
            if (lane == 0) tot[b] = carry;
        }
    } else {
        for (int b = tid; b < nbins; b += blockDim.x) {
            int s0 = 0;
            for (int g = 0; g < nwg; ++g) s0 += d.hist[(int64_t)g * nbins + b];
            tot[b] = s0;
        }
    }
    int li = 1, lb = 0, lo = 0;
    for (int g = tid; g < nwg; g += blockDim.x) {
        li &= d.flags[g] & 1;
        lb |= (d.flags[g] >> 1) & 1;
        lo |= (d.flags[g] >> 2) & 1;
    }
    if (!li) atomicAnd(&s_int, 0);
    if (lb) atomicOr(&s_bad, 1);
    if (lo) atomicOr(&s_ord, 1);
    __syncthreads();
    // exclusive scan over the bins (one wavefront, 64-wide chunks)
    if (tid < 64) {
        int carry = 0;
        for (int c0 = 0; c0 < nbins; c0 += 64) {
            const int b = c0 + tid;
            int v = b < nbins ? tot[b] : 0;
            const int incl = wave_incl_scan(v);
            if (b < nbins) tot[b] = carry + incl - v;
            carry += __shfl(incl, 63, 64);
        }
        if (tid == 0) tot[nbins] = carry;
    }
    __syncthreads();
    for (int b = tid; b <= nbins; b += blockDim.x) d.binoff[b] = tot[b];
    if (staged) {
        for (int e = tid; e < nwg * nbins; e += blockDim.x) {
            const int g = e / nbins, b = e - g * nbins;
            d.off[e] = tot[b] + cnt[b * nwgp + g];
        }
    } else {
        for (int b = tid; b < nbins; b += blockDim.x) {
            int run = tot[b];
            for (int g = 0; g < nwg; ++g) {
                const int c = d.hist[(int64_t)g * nbins + b];
                d.off[(int64_t)g * nbins + b] = run;
                run += c;
            }
        }
    }
    if (tid == 0) {
        const double c = 2.0 * d.fmax;
        const int dg = (s_int && c == rint(c) && c >= 1.0) ? 1 : 0;
        d.diag[0] = dg;
        if (s_bad) atomicOr(a.dev_err, (unsigned)DEVERR_NONFINITE);
        write_hrec(d, s_int != 0, s_bad != 0, s_ord != 0);
    }
}

// K1c: scatter the points into bin order: first cell, offset, the
// pre-phased sample x_n e^{-j 2 pi (f_lo + h df) t_n} in FP64 (pass 1 forms
// each tapered value from it with one rounding) and the sample's index, by
// which pass 1 gathers its taper's values.  Nothing here depends on the
// tapers, so it runs with the binning, while they are still being computed.
template <typename R>
__global__ __launch_bounds__(NT) void k_bin_geo(NuArgs a, NuSeries d0, const NuSeries* D) {
    const NuSeries d = series_of(d0, D);
    const int wg = blockIdx.x;
    if (wg >= d.nwg) return;
    __shared__ int cur[MAX_BINS];
    for (int b = threadIdx.x; b < a.nbins; b += NT) cur[b] = 0;
    __syncthreads();
    R* dels = (R*)d.dels;
    const int64_t n0 = (int64_t)wg * d.ppw;
    for (int j = threadIdx.x; j < d.ppw; j += NT) {
        const int64_t n = n0 + j;
        if (n >= d.N) break;
        Geo g = point_geo(d.t[n], d.x[n], d.f_lo, d.df, a.h, a.nf, a.w);
        const int bin = (g.l0 & (a.N2 - 1)) / a.B;
        const int pos = d.off[(int64_t)wg * a.nbins + bin] + atomicAdd(&cur[bin], 1);
        d.l0s[pos] = g.l0;
        dels[pos] = (R)g.del;
        d.cx[2 * (int64_t)pos] = g.cre;
        d.cx[2 * (int64_t)pos + 1] = g.cim;
        d.perm[pos] = (int)n;
    }
}

// -------------------------------------------------------------- pass 1
constexpr int NT1 = 256;   // threads per pass-1 workgroup
constexpr int MAXSEG = 8;  // column blocks a pass-1 workgroup gathers points from
constexpr int NT2 = 512;   // threads per pass-2 workgroup

// One point as the owners of a tile row read it: s is the grid column of the
// point's first cell relative to the block's first column c0 (negative when
// the support starts left of the block), so the owner of column cb takes tap
// r = cb - s when 0 <= r < w.
template <typename R>
struct SpreadRec {
    int s;
    R del;
    cplx<R> c;
};

// exclusive prefix sum of cnt[0..n) in place, cnt[n] = total (NT1 threads)
template <int N>
__device__ __forceinline__ void scan_counts(int* cnt, int* wtot) {
    constexpr int PER = (N + NT1 - 1) / NT1;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int v[PER];
    int sum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = t * PER + q;
        v[q] = i < N ? cnt[i] : 0;
        sum += v[q];
    }
    const int incl = wave_incl_scan(sum);
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int run = incl - sum;
    for (int i = 0; i < wv; ++i) run += wtot[i];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = t * PER + q;
        if (i < N) cnt[i] = run;
        run += v[q];
    }
    if (t == NT1 - 1) cnt[N] = run;
    __syncthreads();
}

template <typename R, int N1, int B>
// FP32: four waves per SIMD (four workgroups of four waves per compute unit),
// two for the longest columns (N1 = 1024: 64 KB tiles, two per compute unit)
__global__ __launch_bounds__(NT1, sizeof(R) == 4 ? (N1 <= 512 ? 4 : 2) : 1) void k_pass1(NuArgs a, NuSeries d0, const NuSeries* D) {
    const NuSeries d = series_of(d0, D);
    const int nblk = a.N2 / B;
    const int blk = blockIdx.x % nblk;
    const int k = blockIdx.x / nblk;
    if (k >= d.K) return;
    // the column FFTs' intermediate stages use the layout with a gap every 32
    // elements (the tile stays small enough for four workgroups per compute
    // unit)
    constexpr int PSH = N1 >= 64 ? 5 : 0;
    constexpr int LD = N1 + (PSH ? N1 / 32 : 0) + 1;
    constexpr int G = 64 / B;                               // tile rows per wavefront task
    constexpr int TASKS = N1 * B / NT1;                     // tile cells each thread owns
    // points sorted per chunk: the sorted list lives in the tile's storage,
    // which the spread does not touch before its final store
    constexpr int TILE_BYTES = B * LD * (int)sizeof(cplx<R>);
    constexpr int CAP_T = TILE_BYTES / (int)sizeof(SpreadRec<R>) / NT1 * NT1;
    constexpr int CAP = CAP_T < 4 * NT1 ? CAP_T : 4 * NT1;
    constexpr int PPT = CAP / NT1;                          // points per thread per chunk
    static_assert(64 % B == 0 && (N1 * B) % NT1 == 0 && PPT >= 1 && CAP <= 2048 && N1 <= 1024 && B <= 32,
                  "tile split and the packed point keys");
    __shared__ __attribute__((aligned(16))) cplx<R> tile[B * LD];
    __shared__ int rows[N1 + 1];
    __shared__ int wtot[NT1 / 64];
    __shared__ int s_maxrow;   // largest tile row any point reaches
    __shared__ int s_maxrot;   // the same after the rotation by one row
    __shared__ cplx<R> tw[N1];
    SpreadRec<R>* list = reinterpret_cast<SpreadRec<R>*>(tile);
    const int N2 = a.N2, log_N2 = a.log_N2, nf = a.nf, w = a.w;
    const int c0 = blk * B;
    const cplx<R>* tw_g = (const cplx<R>*)a.tw;
    typedef R R2 __attribute__((ext_vector_type(2)));
    const auto* tw_gv = gp((const R2*)a.tw);
    for (int e = threadIdx.x; e <= N1; e += NT1) rows[e] = 0;
    if (threadIdx.x == 0) {
        s_maxrow = -1;
        s_maxrot = -1;
    }
    const R two_over_w = (R)2 / (R)w;
    const R beta = (R)a.beta;
    typedef double D2 __attribute__((ext_vector_type(2)));
    const auto* dels = gp((const R*)d.dels);
    const auto* cxs = gp((const D2*)d.cx);
    const auto* perm = gp((const int*)d.perm);
    const auto* wk = gp(d.w + (int64_t)k * d.N);
    const auto* l0s = gp((const int*)d.l0s);
    // The first loads go out together, branch-free (clamped indices), in the
    // order their values are needed, since they return in issue order: the
    // bin bounds of the window, the FFT twiddles (FP32), and this thread's
    // first two taper values for the sums below.
    // The points of bins blk - lookback .. blk form one flat range of
    // segments, so that every thread's point loads are independent
    // (lookback + 1 <= MAXSEG is checked when the plan is built).
    // (one load per lane: lane q < MAXSEG the start of segment q, lane
    // MAXSEG + q its end; segments past the lookback repeat the last one)
    const auto* binoff = gp((const int*)d.binoff);
    static_assert(2 * MAXSEG <= 64, "segment bounds in one wavefront load");
    int bv;
    {
        const int ln = threadIdx.x & 63;
        const int lq = ln < MAXSEG ? ln : (ln < 2 * MAXSEG ? ln - MAXSEG : 0);
        int bb = blk - (lq <= a.lookback ? lq : a.lookback);
        if (bb < 0) bb += nblk;
        bv = binoff[bb + (ln >= MAXSEG && ln < 2 * MAXSEG ? 1 : 0)];
    }
    // FP32: the length-N1 FFT twiddles are fetched now and stored to LDS
    // after the spread, so that their latency overlaps the point loads (in
    // FP64 the registers held across the spread cost more than they save)
    constexpr bool TW_EARLY = sizeof(R) == 4;
    constexpr int TWP = (N1 + NT1 - 1) / NT1;
    cplx<R> twp[TWP];
    if constexpr (TW_EARLY) {
#pragma unroll
        for (int q = 0; q < TWP; ++q) {
            const int j = threadIdx.x + q * NT1;
            const R2 g = tw_gv[(j < N1 ? j : 0) * a.tws1];
            twp[q] = {g.x, g.y};
        }
    }
    // with E or the F-statistic: this block's shares of sum_n w_k(t_n)^2
    // and sum_n w_k(t_n), over a contiguous range of samples (summed in a
    // fixed order; pass 2 adds the blocks' shares)
    const bool need = d.E || d.F;
    const int64_t per = (d.N + nblk - 1) / nblk;
    const int64_t n0 = (int64_t)blk * per;
    const int64_t n1 = n0 + per < d.N ? n0 + per : d.N;
    const int64_t na = n0 + threadIdx.x, nb = na + NT1;
    const double wa = wk[na < d.N ? na : d.N - 1];
    const double wb = wk[nb < d.N ? nb : d.N - 1];
    // the bounds are uniform: kept in scalar registers
    int sb[MAXSEG], sl[MAXSEG];
    int total = 0;
#pragma unroll
    for (int q = 0; q < MAXSEG; ++q) {
        sb[q] = __builtin_amdgcn_readlane(bv, q);
        sl[q] = q <= a.lookback ? __builtin_amdgcn_readlane(bv, MAXSEG + q) - sb[q] : 0;
        total += sl[q];
    }
    auto locate = [&](int f) {
        int j = -1, r0 = f;
#pragma unroll
        for (int q = 0; q < MAXSEG; ++q) {
            if (j < 0) {
                if (r0 < sl[q]) j = sb[q] + r0;
                else r0 -= sl[q];
            }
        }
        return j;
    };
    // Owner-computes spreading, chunk by chunk (one chunk holds CAP points,
    // normally the whole window): each chunk's points are counting-sorted by
    // the tile row they reach (integer LDS atomics), then every thread sums,
    // in registers, the taps that land on its TASKS cells.  Float atomics on
    // LDS are avoided: they are many times slower than the sort plus a plain
    // store per cell.
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cb = lane % B, rsub = lane / B;
    cplx<R> acc[TASKS];
#pragma unroll
    for (int u = 0; u < TASKS; ++u) acc[u] = {(R)0, (R)0};
    __syncthreads();   // rows[] is zero before the first count
    const int nchunks = (total + CAP - 1) / CAP;
    for (int ch = 0; ch < nchunks; ++ch) {
        // this thread's points of the chunk: all loads first, then the
        // taper's values at the points' sample indices,
        // c = (R)(x_n e^{-j 2 pi (f_lo + h df) t_n} w_k(t_n))
        int pl0[PPT], pn[PPT];
        R pdel[PPT];
        D2 pcx[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int f = ch * CAP + p * NT1 + threadIdx.x;
            pl0[p] = -1;
            pn[p] = -1;
            pdel[p] = (R)0;
            pcx[p] = D2{0.0, 0.0};
            if (f < total) {
                const int j = locate(f);
                pl0[p] = l0s[j];
                pdel[p] = dels[j];
                pcx[p] = cxs[j];
                pn[p] = perm[j];
            }
        }
        cplx<R> pcv[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            pcv[p] = {(R)0, (R)0};
            if (pn[p] >= 0) {
                const double wv = wk[pn[p]];
                pcv[p] = {(R)(pcx[p].x * wv), (R)(pcx[p].y * wv)};
            }
        }
        // target row of each point and its slot in that row, packed as
        // slot << 16 | row << 6 | (s + 16)  (slot < 2048, row < 1024,
        // -16 < s < 32), -1 for a point that reaches no column of the block
        int pk[PPT];
        int mr = -1, mrot = -1;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            pk[p] = -1;
            if (pl0[p] >= 0) {
                int sc = (pl0[p] & (N2 - 1)) - c0;
                if (sc > N2 / 2) sc -= N2;
                else if (sc <= -N2 / 2) sc += N2;
                if (sc < B && sc > -w) {
                    int base = pl0[p] - sc;   // cell of column c0 in the row the taps reach
                    if (base < 0) base += nf;
                    else if (base >= nf) base -= nf;
                    const int row = base >> log_N2;
                    const int slot = atomicAdd(&rows[row], 1);
                    pk[p] = (slot << 16) | (row << 6) | (sc + 16);
                    mr = max(mr, row);
                    mrot = max(mrot, (row + 1) & (N1 - 1));
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            mr = max(mr, __shfl_xor(mr, o, 64));
            mrot = max(mrot, __shfl_xor(mrot, o, 64));
        }
        if (lane == 0 && mr >= 0) {   // one LDS atomic per wavefront
            atomicMax(&s_maxrow, mr);
            atomicMax(&s_maxrot, mrot);
        }
        __syncthreads();
        scan_counts<N1>(rows, wtot);
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            if (pk[p] >= 0) {
                const int at = rows[(pk[p] >> 6) & 1023] + (pk[p] >> 16);
                if (at < CAP) list[at] = {(pk[p] & 63) - 16, pdel[p], pcv[p]};
            }
        }
        __syncthreads();
        // rows past the largest one any point reaches are empty (a test
        // uniform over the wavefront); the point loop is unrolled so that
        // its LDS reads overlap
        const int maxrow = s_maxrow;
#pragma unroll
        for (int u = 0; u < TASKS; ++u) {
            if ((u * (NT1 / 64) + wv) * G > maxrow) continue;
            const int row = (u * (NT1 / 64) + wv) * G + rsub;
            const int beg = rows[row];
            const int end = min(rows[row + 1], CAP);
#pragma unroll 4
            for (int i = beg; i < end; ++i) {
                const SpreadRec<R> rc = list[i];
                const int r = cb - rc.s;
                if ((unsigned)r < (unsigned)w) {
                    const R phi = es_spread<R>(((R)r + rc.del) * two_over_w, beta);
                    acc[u].x += rc.c.x * phi;
                    acc[u].y += rc.c.y * phi;
                }
            }
        }
        __syncthreads();
        if (ch + 1 < nchunks) {
            for (int e = threadIdx.x; e <= N1; e += NT1) rows[e] = 0;
            __syncthreads();
        }
    }
    // Each column enters its FFT rotated by one row (row r at r + 1 mod N1):
    // points whose support wraps below cell 0 reach the last row, which the
    // rotation brings next to the first ones.  The FFT then carries a factor
    // exp(-2 pi i m1 / N1), undone in the four-step twiddle below.  When every
    // rotated row lies in the first N1 / 8, only those are stored and the FFT
    // skips its first stage (which would only repeat them).
    const bool pruned = N1 >= 64 && s_maxrot < N1 / 8;
#pragma unroll
    for (int u = 0; u < TASKS; ++u) {
        const int row = ((u * (NT1 / 64) + wv) * G + rsub + 1) & (N1 - 1);
        if (!pruned || row < N1 / 8) tile[cb * LD + row] = acc[u];
    }
    if constexpr (TW_EARLY) {
#pragma unroll
        for (int q = 0; q < TWP; ++q) {
            const int j = threadIdx.x + q * NT1;
            if (j < N1) tw[j] = twp[q];
        }
    } else {
        for (int j = threadIdx.x; j < N1; j += NT1) tw[j] = tw_g[j * a.tws1];
    }
    __shared__ double s_red[2][NT1 / 64];
    double sq = 0.0, s1 = 0.0;
    if (need) {
        if (na < n1) {
            sq += wa * wa;
            s1 += wa;
        }
        if (nb < n1) {
            sq += wb * wb;
            s1 += wb;
        }
        for (int64_t n = nb + NT1; n < n1; n += NT1) {
            const double wv = wk[n];
            sq += wv * wv;
            s1 += wv;
        }
        sq = wave_sum_to63(sq);
        s1 = wave_sum_to63(s1);
        if (lane == 63) {
            s_red[0][wv] = sq;
            s_red[1][wv] = s1;
        }
    }
    __syncthreads();
    if (need && threadIdx.x == 0) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int i = 0; i < NT1 / 64; ++i) {
            a0 += s_red[0][i];
            a1 += s_red[1][i];
        }
        d.nrm[(int64_t)blk * d.K + k] = a0;
        d.wsp[(int64_t)blk * d.K + k] = a1;
    }
    fft_lds<R, N1, B, NT1, LD, PSH>(tile, tw, 1, pruned);
    // four-step twiddle exp(-2 pi i c m1 / nf), c = c0 + cb, times
    // exp(2 pi i m1 / N1) for the rotation: exp(-2 pi i (c - N2) m1 / nf),
    // then G[k][m1][l2].  A thread keeps one column cb and steps m1 by
    // S = NT1 / B, so its twiddle advances by the fixed factor
    // exp(-2 pi i (c - N2) S / nf): two sine-cosine pairs per thread and a
    // complex product per element, all in FP64 (the product chain adds about
    // IT ulps)
    cplx<R>* out = (cplx<R>*)d.inter + (int64_t)k * nf;
    {
        constexpr int S = NT1 / B, IT = B * N1 / NT1;
        const int cb = threadIdx.x % B, m0 = threadIdx.x / B;
        const int c = c0 + cb;
        const int cr = c + nf - N2;   // c - N2 modulo nf
        const double two_nf = 2.0 / (double)nf;
        const double xt = (double)((cr * m0) & (nf - 1)) * two_nf;
        const double xr = (double)((cr * S) & (nf - 1)) * two_nf;
        double tr = cospi(xt), ti = -sinpi(xt);
        const double fr = cospi(xr), fi = -sinpi(xr);
#pragma unroll 4
        for (int it = 0; it < IT; ++it) {
            const int m1 = m0 + it * S;
            const cplx<R> twv = {(R)tr, (R)ti};
            out[(int64_t)m1 * N2 + c] = cmul(tile[cb * LD + m1], twv);
            const double nr = tr * fr - ti * fi;
            ti = tr * fi + ti * fr;
            tr = nr;
        }
    }
}

// -------------------------------------------------------------- pass 2
// A workgroup owns M consecutive rows m1 and transforms KC tapers at a time
// (KC * M rows in LDS); every output mode is owned by one thread, which
// accumulates sum_k d_k |J_k|^2 across the tapers in a register.
template <typename R, int N2, int M, int KC>
__global__ __launch_bounds__(NT2) void k_pass2(NuArgs a, NuSeries d0, const NuSeries* D) {
    const NuSeries d = series_of(d0, D);
    constexpr int ROWS = KC * M;
    // the FFTs' intermediate stages use the padded layout when the longer
    // rows still fit the LDS of a compute unit
    constexpr bool PAD = ROWS * (N2 + N2 / 8 + 1) * (int)sizeof(cplx<R>) + N2 * (int)sizeof(cplx<R>) <= 160000;
    constexpr int PSH = PAD ? 3 : 0;
    constexpr int LD = PAD ? N2 + N2 / 8 + 1 : N2 + 1;
    constexpr int OUT_IT = (M * (N2 / 2 + 2) + NT2 - 1) / NT2;
    __shared__ cplx<R> rows[ROWS * LD];
    __shared__ cplx<R> tw[N2];
    __shared__ R s_eval;
    __shared__ R s_wk[64];   // W_k(0), for F
    __shared__ R s_sww;
    const int K = d.K, N1 = a.N1, nf = a.nf;
    const int64_t I = a.I, h = a.h;
    // workgroups are dealt to the 8 XCDs in turn; give each XCD a contiguous
    // range of rows so that the P / E lines it writes merge in its own L2
    int bid = blockIdx.x;
    const int nwg = gridDim.x;
    if ((nwg & 7) == 0) bid = (bid & 7) * (nwg >> 3) + (bid >> 3);
    const int m1_0 = bid * M;
    const cplx<R>* tw_g = (const cplx<R>*)a.tw;
    // global address space: plain global loads, which the LDS-only
    // barriers of the FFT do not wait for
    typedef R R2 __attribute__((ext_vector_type(2)));
    const auto* inter = gp((const R2*)d.inter);
    const R* inv_phihat = (const R*)a.inv_phihat;
    R* P = (R*)d.P;
    R* E = (R*)d.E;
    cplx<R>* J = (cplx<R>*)d.J;
    R* Fo = (R*)d.F;
    // the twiddle table is loaded now and stored to LDS once the first
    // rows' loads are in flight too
    constexpr int TWN = (N2 + NT2 - 1) / NT2;
    cplx<R> twr[TWN];
#pragma unroll
    for (int q = 0; q < TWN; ++q) {
        const int j = threadIdx.x + q * NT2;
        twr[q] = j < N2 ? tw_g[j * a.tws2] : cplx<R>{(R)0, (R)0};
    }
    // modes kept: m2 in [0, npos) (i' >= 0) and [m2neg0, N2) (i' < 0)
    int npos = (int)((I - h + N1 - 1) / N1);
    if (npos > N2) npos = N2;
    int m2neg0 = (int)((nf - h) / N1);
    if (m2neg0 < npos) m2neg0 = npos;
    const int nneg = N2 - m2neg0;
    int nout = M * (npos + nneg);
    if (nout > OUT_IT * NT2) nout = OUT_IT * NT2;   // cannot happen for nf >= 2 I
    R acc[OUT_IT], sjj[OUT_IT];
    cplx<R> sjw[OUT_IT];
#pragma unroll
    for (int it = 0; it < OUT_IT; ++it) {
        acc[it] = (R)0;
        sjj[it] = (R)0;
        sjw[it] = {(R)0, (R)0};
    }
    // a group's rows, all loads in flight together (a row never straddles a
    // wavefront: the taper test is uniform per wavefront); the next group's
    // loads are issued before this group's FFTs, so that they arrive while
    // the LDS work runs
    constexpr int LIT = ROWS * N2 / NT2;
    static_assert(ROWS * N2 % NT2 == 0, "pass-2 tile");
    auto load_group = [&](int kc0, cplx<R> (&v)[LIT]) {
        const int nk = K - kc0 < KC ? K - kc0 : KC;
#pragma unroll
        for (int u = 0; u < LIT; ++u) {
            const int e = threadIdx.x + u * NT2;
            const int r = e / N2, l2 = e - r * N2;
            const int kq = r / M, mm = r - kq * M;
            v[u] = {(R)0, (R)0};
            if (kq < nk) {
                const R2 g = inter[(int64_t)(kc0 + kq) * nf + (int64_t)(m1_0 + mm) * N2 + l2];
                v[u] = {g.x, g.y};
            }
        }
    };
    // (registers for two groups only with groups of at most four rows; the
    // larger groups load in place)
    constexpr bool PREF = ROWS <= 4;
    constexpr int LITN = PREF ? LIT : 1;
    cplx<R> v[LIT], vn[LITN];
    if constexpr (PREF) load_group(0, v);
#pragma unroll
    for (int q = 0; q < TWN; ++q) {
        const int j = threadIdx.x + q * NT2;
        if (j < N2) tw[j] = twr[q];
    }
    if (E || Fo) {
        // |w_k|^2 and W_k(0) = sum_n w_k(t_n): pass 1's per-block shares
        // summed in a fixed order (wavefront v takes tapers v, v + 8, ...),
        // while the first rows are on their way
        __shared__ double s_nrm[64], s_wsm[64];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const auto* nrm = gp((const double*)d.nrm);
        const auto* wsp = gp((const double*)d.wsp);
        for (int k = wv; k < K; k += NT2 / 64) {
            double sq = 0.0, s1 = 0.0;
            for (int b = lane; b < a.nbins; b += 64) {
                sq += nrm[(int64_t)b * K + k];
                s1 += wsp[(int64_t)b * K + k];
            }
            sq = wave_sum_to63(sq);
            s1 = wave_sum_to63(s1);
            if (lane == 63) {
                s_nrm[k] = sq;
                s_wsm[k] = s1;
            }
        }
        __syncthreads();
        if (E && threadIdx.x < 64) {
            // D_k = 2 f_max |w_k|^2 when R(B) = 2 f_max I (lane k)
            double e = 0.0;
            const int k = threadIdx.x;
            if (k < K) {
                const double c = 2.0 * d.fmax;
                e = fabs(d.lambda[k] - 2.0 * d.fw * d.lambda[k] / (c * s_nrm[k]));
            }
            for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
            if (threadIdx.x == 0) s_eval = d.diag[0] ? (R)(e / (double)K) : (R)NAN;
        }
        if (Fo && threadIdx.x < 64) {
            // the tapers' DC gains W_k(0) and sum_k W_k(0)^2 (lane k)
            const int k = threadIdx.x;
            const double wk = k < K ? s_wsm[k] : 0.0;
            s_wk[k] = (R)wk;
            double ww = wk * wk;
            for (int o = 32; o > 0; o >>= 1) ww += __shfl_xor(ww, o, 64);
            if (threadIdx.x == 0) s_sww = (R)ww;
        }
    }
    for (int kc0 = 0; kc0 < K; kc0 += KC) {
        const int nk = K - kc0 < KC ? K - kc0 : KC;
        if constexpr (!PREF) load_group(kc0, v);
#pragma unroll
        for (int u = 0; u < LIT; ++u) {
            const int e = threadIdx.x + u * NT2;
            const int r = e / N2, l2 = e - r * N2;
            rows[r * LD + l2] = v[u];
        }
        __syncthreads();
        if constexpr (PREF) {
            if (kc0 + KC < K) load_group(kc0 + KC, vn);
        }
        fft_lds<R, N2, ROWS, NT2, LD, PSH>(rows, tw, 1, false, nk * M);   // the nk tapers present
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
                    const R sc = inv_phihat[kk < 0 ? -kk : kk];
                    for (int kq = 0; kq < nk; ++kq) {
                        const cplx<R> v = cscale(rows[(kq * M + mm) * LD + m2], sc);
                        const R dd = d.dk ? (R)d.dk[kc0 + kq] : (R)1 / (R)K;
                        const R vv = v.x * v.x + v.y * v.y;
                        acc[it] += dd * vv;
                        if (J) J[(int64_t)(kc0 + kq) * I + i] = v;
                        if (Fo) {
                            const R wk = s_wk[kc0 + kq];
                            sjw[it].x += v.x * wk;
                            sjw[it].y += v.y * wk;
                            sjj[it] += vv;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if constexpr (PREF) {
#pragma unroll
            for (int u = 0; u < LIT; ++u) v[u] = vn[u];
        }
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
                if (Fo) Fo[i] = f_statistic<R>(sjw[it], sjj[it], s_sww, K);
            }
        }
    }
}

// Pass 2 with wavefront-private row transforms: a workgroup owns one row m1
// and its eight wavefronts take the tapers in turn (wavefront v: tapers v,
// v + 8, ...); each transforms its row alone (wave_fft: no workgroup
// barrier between stages) and accumulates d_k |J_k|^2 for the 16 modes
// l + 64 m its lane holds.  The wavefronts' sums are added in a fixed order
// at the end.  Rows of N2 = 512, 1024 or 2048 (FP32 only), P and E only
// (batches that ask for the eigencoefficients or the F-statistic take the
// general kernel); FP32 rows up to 1024 with four waves per SIMD, the rest
// with two (152-156 KB of LDS at the largest rows).
template <typename R, int N2>
__global__ __launch_bounds__(NT2, sizeof(R) == 4 && N2 <= 1024 ? 4 : 2) void k_pass2w(NuArgs a, NuSeries d0, const NuSeries* D) {
    const NuSeries d = series_of(d0, D);
    using W = WavePlan<N2>;
    using T = WaveTw<N2>;
    constexpr int E = W::E, WLD = N2 + (N2 >> W::PSH), NW = NT2 / 64;
    static_assert(NW * N2 * sizeof(R) <= NW * WLD * sizeof(cplx<R>), "sums fit the transform space");
    __shared__ __attribute__((aligned(16))) cplx<R> wbuf[NW * WLD];
    __shared__ cplx<R> twt[T::NB + T::NC];
    __shared__ R s_eval;
    const int K = d.K, N1 = a.N1, nf = a.nf;
    const int64_t I = a.I, h = a.h;
    // rows dealt to the 8 XCDs in contiguous ranges, as in k_pass2
    int bid = blockIdx.x;
    const int nwg = gridDim.x;
    if ((nwg & 7) == 0) bid = (bid & 7) * (nwg >> 3) + (bid >> 3);
    const int m1 = bid;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    typedef R R2 __attribute__((ext_vector_type(2)));
    const auto* inter = gp((const R2*)d.inter);
    const auto* tw_g = gp((const R2*)a.tw);
    const R* inv_phihat = (const R*)a.inv_phihat;
    R* P = (R*)d.P;
    R* Ep = (R*)d.E;
    cplx<R> v[E];
    auto load_row = [&](int k) {
        const auto* src = inter + (int64_t)k * nf + (int64_t)m1 * N2 + lane;
#pragma unroll
        for (int t = 0; t < E; ++t) {
            const R2 g = src[64 * t];
            v[t] = {g.x, g.y};
        }
    };
    // Every load is issued up front, branch-free (a clamped index or a valid
    // stand-in address), in the order the values are needed: loads return in
    // issue order, so the twiddle table and E can be finished while the row
    // is still on its way.  Pass 1's shares of |w_k|^2 are preloaded when
    // each wavefront has one taper and there are at most 64 NQ blocks.
    constexpr int NQ = N2 >= 2048 ? 4 : 2;
    const auto* nrm = gp((const double*)d.nrm);
    const bool pre = K <= NW && a.nbins <= 64 * NQ;
    const int kw = wv < K ? wv : K - 1;
    double nq[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) nq[u] = nrm[(int64_t)(lane + 64 * u < a.nbins ? lane + 64 * u : 0) * K + kw];
    const double lam = gp(d.lambda ? d.lambda : (const double*)d.nrm)[lane < K ? lane : 0];
    const int diag = gp((const int*)d.diag)[0];
    const double dkv = gp(d.dk ? d.dk : (const double*)d.nrm)[kw];
    constexpr int TWR = (T::NB + T::NC + NT2 - 1) / NT2;
    cplx<R> twr[TWR];
#pragma unroll
    for (int q = 0; q < TWR; ++q) {
        const int e = threadIdx.x + q * NT2;
        const R2 g = tw_g[T::index(e < T::NB + T::NC ? e : 0) * a.tws2];
        twr[q] = {g.x, g.y};
    }
    load_row(kw);
#pragma unroll
    for (int q = 0; q < TWR; ++q) {
        const int e = threadIdx.x + q * NT2;
        if (e < T::NB + T::NC) twt[e] = twr[q];
    }
    if (Ep) {
        // D_k = 2 f_max |w_k|^2 when R(B) = 2 f_max I: |w_k|^2 from pass 1's
        // per-block shares, summed in a fixed order (wavefront v takes
        // tapers v, v + 8, ...)
        __shared__ double s_nrm[64];
        if (pre) {
            double sq = 0.0;
#pragma unroll
            for (int u = 0; u < NQ; ++u) sq += lane + 64 * u < a.nbins ? nq[u] : 0.0;
            sq = wave_sum_to63(sq);
            if (lane == 63 && wv < K) s_nrm[wv] = sq;
        } else {
            for (int k = wv; k < K; k += NW) {
                double sq = 0.0;
                for (int b = lane; b < a.nbins; b += 64) sq += nrm[(int64_t)b * K + k];
                sq = wave_sum_to63(sq);
                if (lane == 63) s_nrm[k] = sq;
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            double e = 0.0;
            const int k = threadIdx.x;
            if (k < K) {
                const double c = 2.0 * d.fmax;
                e = fabs(lam - 2.0 * d.fw * lam / (c * s_nrm[k]));
            }
            for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
            if (threadIdx.x == 0) s_eval = diag ? (R)(e / (double)K) : (R)NAN;
        }
    }
    __syncthreads();   // twiddle table
    // modes kept: m2 in [0, npos) (i' >= 0) and [m2neg0, N2) (i' < 0)
    int npos = (int)((I - h + N1 - 1) / N1);
    if (npos > N2) npos = N2;
    int m2neg0 = (int)((nf - h) / N1);
    if (m2neg0 < npos) m2neg0 = npos;
    R acc[E];
#pragma unroll
    for (int m = 0; m < E; ++m) acc[m] = (R)0;
    cplx<R>* wb = wbuf + wv * WLD;
    for (int k = wv; k < K; k += NW) {
        if (k != wv) load_row(k);
        wave_fft<R, N2>(v, wb, twt);
        const R dd = d.dk ? (R)(k == wv ? dkv : d.dk[k]) : (R)1 / (R)K;
#pragma unroll
        for (int m = 0; m < E; ++m) acc[m] += dd * (v[m].x * v[m].x + v[m].y * v[m].y);
    }
    __syncthreads();   // every wavefront is done with its region
    R* red = reinterpret_cast<R*>(wbuf);
#pragma unroll
    for (int m = 0; m < E; ++m) red[wv * N2 + lane + 64 * m] = acc[m];
    __syncthreads();
    for (int m2 = threadIdx.x; m2 < N2; m2 += NT2) {
        if (!(m2 < npos || m2 >= m2neg0)) continue;
        const int64_t mm = (int64_t)m1 + (int64_t)N1 * m2;
        const int64_t kk = mm < nf / 2 ? mm : mm - nf;
        const int64_t i = kk + h;
        if (i < 0 || i >= I) continue;
        R sum = (R)0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sum += red[w * N2 + m2];
        const R sc = inv_phihat[kk < 0 ? -kk : kk];
        if (P) P[i] = sum * (sc * sc);
        if (Ep) Ep[i] = s_eval;
    }
}

// ------------------------------------------------- single-workgroup path
template <typename R, int NF>
__global__ __launch_bounds__(NT) void k_small(NuArgs a, NuSeries d0, const NuSeries* D) {
    const NuSeries d = series_of(d0, D);
    constexpr int OUT_IT = (NF / 2 + NT - 1) / NT;
    __shared__ cplx<R> grid[NF];
    __shared__ double red[NT / 64];
    __shared__ int s_int, s_bad, s_ord;
    if (threadIdx.x == 0) {
        s_int = 1;
        s_bad = 0;
        s_ord = 0;
    }
    const int K = d.K, w = a.w;
    const int64_t I = a.I, h = a.h, N = d.N;
    const cplx<R>* tw = (const cplx<R>*)a.tw;
    const R* inv_phihat = (const R*)a.inv_phihat;
    R* P = (R*)d.P;
    R* E = (R*)d.E;
    cplx<R>* J = (cplx<R>*)d.J;
    R* Fo = (R*)d.F;
    R acc[OUT_IT], sjj[OUT_IT];
    cplx<R> sjw[OUT_IT];
#pragma unroll
    for (int it = 0; it < OUT_IT; ++it) {
        acc[it] = (R)0;
        sjj[it] = (R)0;
        sjw[it] = {(R)0, (R)0};
    }
    const R two_over_w = (R)2 / (R)w;
    const R beta = (R)a.beta;
    double esum = 0.0, sww = 0.0;
    for (int k = 0; k < K; ++k) {
        for (int e = threadIdx.x; e < NF; e += NT) grid[e] = {(R)0, (R)0};
        __syncthreads();
        const double* wk = d.w + (int64_t)k * N;
        double nrm = 0.0, wsum = 0.0;
        int my_int = 1, my_bad = 0, my_ord = 0;
        for (int64_t n = threadIdx.x; n < N; n += NT) {
            const double tn = d.t[n];
            const Geo g = point_geo(tn, d.x[n], d.f_lo, d.df, h, NF, w);
            my_int &= g.integral ? 1 : 0;
            my_bad |= g.ok ? 0 : 1;
            if (k == 0 && d.hrec && n > 0 && !(tn > d.t[n - 1])) my_ord = 1;
            const double wv = wk[n];
            nrm += wv * wv;
            wsum += wv;
            const cplx<R> c = {(R)(g.cre * wv), (R)(g.cim * wv)};
            const R del = (R)g.del;
            for (int r = 0; r < w; ++r) {
                int cell = g.l0 + r;
                if (cell >= NF) cell -= NF;
                const R phi = es_spread<R>(((R)r + del) * two_over_w, beta);
                atomicAdd(&grid[cell].x, c.x * phi);
                atomicAdd(&grid[cell].y, c.y * phi);
            }
        }
        if (!my_int) atomicAnd(&s_int, 0);
        if (my_bad) atomicOr(&s_bad, 1);
        if (my_ord) atomicOr(&s_ord, 1);
        nrm = block_sum(nrm, red);   // contains barriers
        if (Fo) {
            wsum = block_sum(wsum, red);   // W_k(0), the taper's DC gain
            sww += wsum * wsum;
        }
        if (E && d.lambda) {
            const double c = 2.0 * d.fmax;
            esum += fabs(d.lambda[k] - 2.0 * d.fw * d.lambda[k] / (c * nrm));
        }
        fft_lds<R, NF, 1, NT, NF>(grid, tw, a.tws1);
        const R dd = d.dk ? (R)d.dk[k] : (R)1 / (R)K;
#pragma unroll
        for (int it = 0; it < OUT_IT; ++it) {
            const int64_t i = threadIdx.x + (int64_t)it * NT;
            if (i < I) {
                const int64_t kk = i - h;
                const int64_t m = kk < 0 ? kk + NF : kk;
                const R sc = inv_phihat[kk < 0 ? -kk : kk];
                const cplx<R> v = cscale(grid[m], sc);
                const R vv = v.x * v.x + v.y * v.y;
                acc[it] += dd * vv;
                if (J) J[(int64_t)k * I + i] = v;
                if (Fo) {
                    sjw[it].x += v.x * (R)wsum;
                    sjw[it].y += v.y * (R)wsum;
                    sjj[it] += vv;
                }
            }
        }
        __syncthreads();
    }
    const double c = 2.0 * d.fmax;
    const bool diag = s_int && c == rint(c) && c >= 1.0;
    const R ev = diag ? (R)(esum / (double)K) : (R)NAN;
    if (threadIdx.x == 0) {
        if (s_bad) atomicOr(a.dev_err, (unsigned)DEVERR_NONFINITE);
        write_hrec(d, s_int != 0, s_bad != 0, s_ord != 0);
    }
#pragma unroll
    for (int it = 0; it < OUT_IT; ++it) {
        const int64_t i = threadIdx.x + (int64_t)it * NT;
        if (i < I) {
            if (P) P[i] = acc[it];
            if (E) E[i] = ev;
            if (Fo) Fo[i] = f_statistic<R>(sjw[it], sjj[it], (R)sww, K);
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
        NuSchedule sch;
        auto si = ctx->schedule.find(std::make_tuple(p.I, p.prec, p.w));
        if (si != ctx->schedule.end()) sch = si->second;
        int L = p.log_nf;
        int l1 = L / 2;
        if (l1 > 10) l1 = 10;
        if (sch.l1 > 0) l1 = sch.l1;
        p.N1 = 1 << l1;
        p.N2 = p.nf / p.N1;
        if (p.N2 > 4096) {
            set_error("band count too large for this build (nf = %d)", p.nf);
            return M2N_ERR_UNSUPPORTED;
        }
        // pass 1: B columns of N1 values per workgroup, a 32 KB tile (four
        // workgroups per compute unit; narrow blocks waste fewer lanes of
        // the spread, whose points cover w of the B columns).  B >= 8 in
        // FP32 and >= 4 in FP64: narrower blocks multiply the bins of the
        // counting sort (measured slower at N1 = 1024)
        p.B = 32768 / (p.N1 * cs);
        if (p.B > 32) p.B = 32;
        if (p.B > p.N2 / 2) p.B = p.N2 / 2;
        if (p.B < 8 && sizeof(R) == 4) p.B = 8;
        if (p.B < 4) p.B = 4;
        if (sch.B > 0) p.B = sch.B;
        p.lookback = (p.w - 1 + p.B - 1) / p.B;
        if (p.lookback >= p.N2 / p.B || p.N2 / p.B > MAX_BINS || p.lookback + 1 > MAXSEG) {
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
        if (sch.M > 0) p.M_force = sch.M;
        Nt = p.N1 > p.N2 ? p.N1 : p.N2;
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

int width_of(int prec, double tol) {
    if (tol <= 0.0) tol = (prec == M2N_FP32) ? 1e-6 : 1e-12;
    int w = (int)std::ceil(-std::log10(tol)) + 1;
    if (w < 4) w = 4;
    if (prec == M2N_FP32 && w > 8) w = 8;
    if (w > 16) w = 16;
    return w;
}

int get_plan(Ctx* ctx, int64_t I, int prec, double tol, NufftPlan** out) {
    const int w = width_of(prec, tol);
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
        ctx->release(p->inv_phihat);
        return st;
    }
    *out = p.get();
    ctx->plans.emplace(key, std::move(p));
    return M2N_OK;
}

// ---------------------------------------------------------- dispatchers

NuArgs make_args(Ctx* ctx, const NufftPlan& p) {
    NuArgs a{};
    a.I = p.I;
    a.h = p.h;
    a.beta = p.beta;
    a.nf = p.nf;
    a.w = p.w;
    a.N1 = p.N1;
    a.N2 = p.N2;
    a.B = p.B;
    a.nbins = p.single ? 0 : p.N2 / p.B;
    a.log_N2 = p.single ? 0 : ilog2i(p.N2);
    a.lookback = p.lookback;
    a.tws1 = p.single ? 1 : p.tw_len / p.N1;
    a.tws2 = p.single ? 1 : p.tw_len / p.N2;
    a.tw = p.tw_fft.p;
    a.inv_phihat = p.inv_phihat.p;
    a.dev_err = ctx->dev_err;
    return a;
}

template <typename R>
int launch_small(const NufftPlan& p, hipStream_t st, dim3 grid, const NuArgs& a, const NuSeries& d0,
                 const NuSeries* D) {
#define M2N_SMALL(NFV)                                                                       \
    case NFV:                                                                                \
        hipLaunchKernelGGL((k_small<R, NFV>), grid, dim3(NT), 0, st, a, d0, D);            \
        return M2N_OK;
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
    set_error("no single-workgroup kernel for nf = %d", p.nf);
    return M2N_ERR_UNSUPPORTED;
}

template <typename R>
int launch_pass1(const NufftPlan& p, hipStream_t st, dim3 grid, const NuArgs& a, const NuSeries& d0,
                 const NuSeries* D) {
#define M2N_P1(N1V, BV)                                                                    \
    if (p.N1 == N1V && p.B == BV) {                                                        \
        hipLaunchKernelGGL((k_pass1<R, N1V, BV>), grid, dim3(NT1), 0, st, a, d0, D);       \
        return M2N_OK;                                                                     \
    }
    if constexpr (sizeof(R) == 4) {
        M2N_P1(64, 32) M2N_P1(128, 32) M2N_P1(256, 16) M2N_P1(512, 8) M2N_P1(1024, 8)
        M2N_P1(256, 8) M2N_P1(512, 16)
    } else {
        M2N_P1(64, 32) M2N_P1(128, 16) M2N_P1(256, 8) M2N_P1(512, 4) M2N_P1(1024, 4)
        M2N_P1(256, 4) M2N_P1(512, 8)
    }
#undef M2N_P1
    set_error("no pass-1 kernel for N1 = %d, B = %d", p.N1, p.B);
    return M2N_ERR_UNSUPPORTED;
}

// rows-per-workgroup choice for pass 2: largest M the LDS budget allows that
// still gives at least two workgroups per compute unit (counting a batch)
inline int pass2_rows(const NufftPlan& p, int cu_count, int nseries) {
    if (p.M_force > 0) return p.M_force;
    int M = p.M;
    while (M > 1 && (int64_t)(p.N1 / M) * nseries < 2 * cu_count) M /= 2;
    return M;
}

// Taper group of a pass-2 launch: with one row per workgroup and more than
// four tapers, groups of four (half the LDS of eight, so more workgroups per
// compute unit, and a second group whose loads overlap the first group's
// FFTs); else the plan's.
inline int pass2_group(const NufftPlan& p, int M, int maxK) { return M == 1 && maxK > 4 && p.KC > 4 ? 4 : p.KC; }

template <typename R>
int launch_pass2(const NufftPlan& p, hipStream_t st, int M, int KC, dim3 grid, const NuArgs& a,
                 const NuSeries& d0, const NuSeries* D) {
#define M2N_P2(N2V, MV, KCV)                                                               \
    if (p.N2 == N2V && M == MV && KC == KCV) {                                             \
        hipLaunchKernelGGL((k_pass2<R, N2V, MV, KCV>), grid, dim3(NT2), 0, st, a, d0, D);  \
        return M2N_OK;                                                                     \
    }
    if constexpr (sizeof(R) == 4) {
        M2N_P2(128, 1, 8) M2N_P2(128, 2, 8) M2N_P2(128, 4, 8)
        M2N_P2(256, 1, 8) M2N_P2(256, 2, 8) M2N_P2(256, 4, 8)
        M2N_P2(512, 1, 8) M2N_P2(512, 2, 8) M2N_P2(512, 4, 8)
        M2N_P2(1024, 1, 8) M2N_P2(1024, 2, 8)
        M2N_P2(2048, 1, 8) M2N_P2(4096, 1, 2)
        M2N_P2(128, 1, 4) M2N_P2(256, 1, 4) M2N_P2(512, 1, 4) M2N_P2(1024, 1, 4) M2N_P2(2048, 1, 4)
    } else {
        M2N_P2(128, 1, 8) M2N_P2(128, 2, 8) M2N_P2(128, 4, 8)
        M2N_P2(256, 1, 8) M2N_P2(256, 2, 8) M2N_P2(256, 4, 8)
        M2N_P2(512, 1, 8) M2N_P2(512, 2, 8)
        M2N_P2(1024, 1, 8) M2N_P2(2048, 1, 2) M2N_P2(4096, 1, 1)
        M2N_P2(128, 1, 4) M2N_P2(256, 1, 4) M2N_P2(512, 1, 4) M2N_P2(1024, 1, 4)
    }
#undef M2N_P2
    set_error("no pass-2 kernel for N2 = %d, M = %d, KC = %d", p.N2, M, KC);
    return M2N_ERR_UNSUPPORTED;
}

// 256-byte aligned carving of one workspace
struct Carver {
    char* base = nullptr;
    size_t used = 0;
    void* take(size_t bytes) {
        void* p = base ? base + used : nullptr;
        used += (bytes + 255) & ~size_t(255);
        return p;
    }
};

// `checked` (or NULL) is recorded once the kernels that write the series'
// host records of the t check (k_scan, k_small) are queued
}  // namespace

// A NuFFT batch whose binning (histogram and scan of the cells, which need
// t alone) is queued and whose scatter, passes and outputs are not: the
// tapers may still be in flight between the two halves.
struct NuPending {
    const NufftPlan* p = nullptr;
    int prec = 0;
    NuArgs a{};
    std::vector<NuSeries> ds;
    const NuSeries* D = nullptr;
    int maxK = 0, maxwg = 0;
};

namespace {

template <typename R>
int begin_typed(Ctx* ctx, hipStream_t st, const NufftPlan& p, const NuSeriesIn* in, int ns, NuPending& q) {
    q.p = &p;
    q.a = make_args(ctx, p);
    std::vector<NuSeries>& ds = q.ds;
    ds.assign(ns, NuSeries());
    int maxK = 0, maxwg = 0;
    // per-series binning geometry, then the workspace layout (two passes:
    // measure with a null base, then carve)
    const int nbins = p.single ? 0 : p.N2 / p.B;
    for (int i = 0; i < ns; ++i) {
        NuSeries& d = ds[i];
        std::memset(&d, 0, sizeof(d));
        const NuSeriesIn& s = in[i];
        d.t = s.t;
        d.x = s.x;
        d.w = s.w;
        d.lambda = s.lambda;
        d.dk = s.dk;
        d.P = s.P;
        d.E = s.E;
        d.J = s.J;
        d.F = s.F;
        d.hrec = s.hrec;
        d.N = s.N;
        d.f_lo = s.f_lo;
        d.df = s.df;
        d.fmax = s.fmax;
        d.fw = s.fw;
        d.K = s.K;
        if (!p.single) {
            // points per binning workgroup: one per thread unless the scan
            // could then not stage every (workgroup, bin) count in LDS
            int64_t ppw = NT;
            while ((s.N + ppw - 1) / ppw * nbins > SCAN_LDS && ppw < (int64_t(1) << 20)) ppw *= 2;
            const int64_t nwg64 = (s.N + ppw - 1) / ppw;
            if (nwg64 > (1 << 20)) {
                set_error("N too large");
                return M2N_ERR_ARG;
            }
            d.ppw = (int)ppw;
            d.nwg = (int)nwg64;
        }
        maxK = std::max(maxK, s.K);
        maxwg = std::max(maxwg, d.nwg);
    }
    q.maxK = maxK;
    q.maxwg = maxwg;
    if (!p.single) {
        auto carve = [&](Carver& c) {
            for (int i = 0; i < ns; ++i) {
                NuSeries& d = ds[i];
                const size_t N = (size_t)d.N;
                d.hist = (int*)c.take(sizeof(int) * (size_t)d.nwg * nbins);
                d.off = (int*)c.take(sizeof(int) * (size_t)d.nwg * nbins);
                d.binoff = (int*)c.take(sizeof(int) * (size_t)(nbins + 1));
                d.flags = (int*)c.take(sizeof(int) * (size_t)d.nwg);
                d.l0s = (int*)c.take(sizeof(int) * N);
                d.dels = c.take(sizeof(R) * N);
                d.cx = (double*)c.take(2 * sizeof(double) * N);
                d.perm = (int*)c.take(sizeof(int) * N);
                d.inter = c.take(sizeof(cplx<R>) * (size_t)d.K * p.nf);
                d.nrm = (double*)c.take(sizeof(double) * (size_t)nbins * d.K);
                d.wsp = (double*)c.take(sizeof(double) * (size_t)nbins * d.K);
                d.diag = (int*)c.take(64);
            }
        };
        Carver m;
        carve(m);
        void* wsp;
        M2N_TRY(ctx->workspace("nu_work", m.used, &wsp));
        Carver c;
        c.base = (char*)wsp;
        carve(c);
    }
    q.D = nullptr;
    if (ns > 1) {
        void* vd;
        M2N_TRY(ctx->workspace("nu_desc", sizeof(NuSeries) * (size_t)ns, &vd));
        M2N_TRY(ctx->stage(st, ds.data(), sizeof(NuSeries) * (size_t)ns, vd));
        q.D = (const NuSeries*)vd;
    }
    if (p.single) return M2N_OK;
    const NuSeries& d0 = ds[0];
    const unsigned ys = (unsigned)ns;
    {
        M2N_PROF(ctx, st, "k_hist");
        hipLaunchKernelGGL(k_hist, dim3((unsigned)maxwg, ys), dim3(NT), 0, st, q.a, d0, q.D);
    }
    {
        M2N_PROF(ctx, st, "k_scan");
        hipLaunchKernelGGL(k_scan, dim3(1, ys), dim3(1024), 0, st, q.a, d0, q.D);
    }
    {
        M2N_PROF(ctx, st, "k_bin_geo");
        hipLaunchKernelGGL(k_bin_geo<R>, dim3((unsigned)maxwg, ys), dim3(NT), 0, st, q.a, d0, q.D);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

// the second half: scatter, the two passes (or the one-workgroup kernel for
// small grids); `checked` (if given) is recorded once the t check of the
// binning is done
template <typename R>
int finish_typed(Ctx* ctx, hipStream_t st, NuPending& q, hipEvent_t checked) {
    const NufftPlan& p = *q.p;
    const NuSeries& d0 = q.ds[0];
    const NuSeries* D = q.D;
    const int ns = (int)q.ds.size();
    const unsigned ys = (unsigned)ns;
    if (p.single) {
        M2N_PROF(ctx, st, "k_small");
        M2N_TRY(launch_small<R>(p, st, dim3(1, ys), q.a, d0, D));
        M2N_HIP(hipGetLastError());
        if (checked) M2N_HIP(hipEventRecord(checked, st));
        return M2N_OK;
    }
    const int nbins = p.N2 / p.B;
    if (checked) M2N_HIP(hipEventRecord(checked, st));
    {
        M2N_PROF(ctx, st, "k_pass1");
        M2N_TRY(launch_pass1<R>(p, st, dim3((unsigned)(q.maxK * nbins), ys), q.a, d0, D));
    }
    M2N_HIP(hipGetLastError());
    {
        M2N_PROF(ctx, st, "k_pass2");
        const int M = pass2_rows(p, ctx->cu_count, ns);
        bool anyJF = false;
        for (const NuSeries& d : q.ds) anyJF = anyJF || d.F != nullptr || d.J != nullptr;
        bool wave_rows = false;
        // P and E only, rows of 512 or 1024: wavefront-private row FFTs, one
        // row per workgroup (unless a tuned schedule fixed the rows)
        // (rows of 2048 in FP32 only: the FP64 regions exceed the LDS)
        if ((M == 1 || p.M_force == 0) && !anyJF &&
            (p.N2 == 512 || p.N2 == 1024 || (p.N2 == 2048 && sizeof(R) == 4))) {
            wave_rows = true;
            if (p.N2 == 1024) hipLaunchKernelGGL((k_pass2w<R, 1024>), dim3((unsigned)p.N1, ys), dim3(NT2), 0, st, q.a, d0, D);
            else if (p.N2 == 512) hipLaunchKernelGGL((k_pass2w<R, 512>), dim3((unsigned)p.N1, ys), dim3(NT2), 0, st, q.a, d0, D);
            else if constexpr (sizeof(R) == 4) hipLaunchKernelGGL((k_pass2w<R, 2048>), dim3((unsigned)p.N1, ys), dim3(NT2), 0, st, q.a, d0, D);
        }
        if (!wave_rows)
            M2N_TRY(launch_pass2<R>(p, st, M, pass2_group(p, M, q.maxK), dim3((unsigned)(p.N1 / M), ys), q.a, d0, D));
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

template <typename R>
int run_typed(Ctx* ctx, hipStream_t st, const NufftPlan& p, const NuSeriesIn* in, int ns, hipEvent_t checked) {
    NuPending q;
    M2N_TRY(begin_typed<R>(ctx, st, p, in, ns, q));
    return finish_typed<R>(ctx, st, q, checked);
}

int check_series(const NuSeriesIn& s, int64_t I) {
    if (!s.t || !s.x || !s.w || s.N < 1 || s.K < 1 || s.K > 64 || I < 1 ||
        I > (int64_t(1) << 21)) {
        set_error("bad argument (N = %lld, K = %d, I = %lld)", (long long)s.N, s.K, (long long)I);
        return M2N_ERR_ARG;
    }
    if (s.N > (int64_t(1) << 30)) {
        set_error("N too large");
        return M2N_ERR_ARG;
    }
    if (!std::isfinite(s.f_lo) || !std::isfinite(s.df) || !(s.df > 0.0)) {
        set_error("band grid must have finite f_lo and df > 0");
        return M2N_ERR_ARG;
    }
    if (s.E && (!s.lambda || !(s.fmax > 0.0) || !(s.fw > 0.0))) {
        set_error("E needs lambda, fmax > 0 and fw > 0");
        return M2N_ERR_ARG;
    }
    if (s.F && s.K < 2) {
        set_error("the F-statistic needs K >= 2 tapers (F(2, 2K-2))");
        return M2N_ERR_ARG;
    }
    return M2N_OK;
}

}  // namespace

int nufft_run_batch(Ctx* ctx, hipStream_t st, int64_t I, int prec, double tol,
                    const NuSeriesIn* series, int nseries) {
    if (nseries < 1 || !series) {
        set_error("empty batch");
        return M2N_ERR_ARG;
    }
    if (prec != M2N_FP32 && prec != M2N_FP64) {
        set_error("prec must be M2N_FP32 or M2N_FP64");
        return M2N_ERR_ARG;
    }
    for (int i = 0; i < nseries; ++i) M2N_TRY(check_series(series[i], I));
    NufftPlan* p = nullptr;
    M2N_TRY(get_plan(ctx, I, prec, tol, &p));
    // Ehat: where R(B) is a multiple of the identity the NuFFT pass writes
    // it (band-constant); elsewhere the window quadrature overwrites it.  The
    // binning kernels record what they saw of t in pinned host memory; the
    // host reads it once the whole NuFFT is queued, so the device does not
    // wait for the host.
    std::vector<int> eidx;
    for (int i = 0; i < nseries; ++i)
        if (series[i].E && !series[i].e_diag_known) eidx.push_back(i);
    if (eidx.empty()) {
        if (prec == M2N_FP32) return run_typed<float>(ctx, st, *p, series, nseries, nullptr);
        return run_typed<double>(ctx, st, *p, series, nseries, nullptr);
    }
    M2N_TRY(ctx->pinned_erec((size_t)nseries * 4 * sizeof(double)));
    double* rec = (double*)ctx->erec;
    std::vector<NuSeriesIn> ser(series, series + nseries);
    for (int i : eidx) {
        ser[i].hrec = rec + 4 * i;
        rec[4 * i] = -1.0;
    }
    if (!ctx->tcheck_ev) M2N_HIP(hipEventCreateWithFlags(&ctx->tcheck_ev, hipEventDisableTiming));
    if (prec == M2N_FP32) M2N_TRY(run_typed<float>(ctx, st, *p, ser.data(), nseries, ctx->tcheck_ev));
    else M2N_TRY(run_typed<double>(ctx, st, *p, ser.data(), nseries, ctx->tcheck_ev));
    M2N_HIP(hipEventSynchronize(ctx->tcheck_ev));
    for (int i : eidx) {
        const NuSeriesIn& s = series[i];
        const double* r = rec + 4 * i;
        const int flags = (int)r[0];
        if (flags < 0) {
            set_error("series %d: the t check left no record", i);
            return M2N_ERR_HIP;
        }
        if (flags & 1) continue;   // non-finite t: reported by m2n_check
        if (flags & 2) {
            set_error("series %d: Ehat needs strictly increasing sampling times", i);
            return M2N_ERR_T_ORDER;
        }
        const double c = 2.0 * s.fmax;
        const bool diag = !(flags & 4) && c == std::rint(c) && c >= 1.0;
        if (!diag) M2N_TRY(ehat_general(ctx, st, I, prec, tol, s, s.N > 1 ? r[2] - r[1] : 0.0));
    }
    return M2N_OK;
}

int nufft_begin(Ctx* ctx, hipStream_t st, int64_t I, int prec, double tol, const NuSeriesIn* series,
                int nseries, NuPending** out) {
    *out = nullptr;
    if (nseries < 1 || !series) {
        set_error("empty batch");
        return M2N_ERR_ARG;
    }
    if (prec != M2N_FP32 && prec != M2N_FP64) {
        set_error("prec must be M2N_FP32 or M2N_FP64");
        return M2N_ERR_ARG;
    }
    for (int i = 0; i < nseries; ++i) {
        M2N_TRY(check_series(series[i], I));
        if (series[i].E && !series[i].e_diag_known) {
            set_error("series %d: a split NuFFT needs Ehat routed by its caller", i);
            return M2N_ERR_ARG;
        }
    }
    NufftPlan* p = nullptr;
    M2N_TRY(get_plan(ctx, I, prec, tol, &p));
    std::unique_ptr<NuPending> q(new NuPending());
    q->prec = prec;
    if (prec == M2N_FP32) M2N_TRY(begin_typed<float>(ctx, st, *p, series, nseries, *q));
    else M2N_TRY(begin_typed<double>(ctx, st, *p, series, nseries, *q));
    *out = q.release();
    return M2N_OK;
}

int nufft_finish(Ctx* ctx, hipStream_t st, NuPending* q) {
    std::unique_ptr<NuPending> own(q);
    if (q->prec == M2N_FP32) return finish_typed<float>(ctx, st, *q, nullptr);
    return finish_typed<double>(ctx, st, *q, nullptr);
}

void nufft_pending_free(NuPending* q) { delete q; }

int nufft_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N,
              const double* w, int K, double f_lo, double df, int64_t I, int prec, double tol,
              const double* weights, const double* lambda, double fmax, double fw, void* P,
              void* E, void* J, void* F) {
    NuSeriesIn s;
    s.t = t;
    s.x = x;
    s.w = w;
    s.lambda = lambda;
    s.dk = weights;
    s.N = N;
    s.K = K;
    s.f_lo = f_lo;
    s.df = df;
    s.fmax = fmax;
    s.fw = fw;
    s.P = P;
    s.E = E;
    s.J = J;
    s.F = F;
    return nufft_run_batch(ctx, st, I, prec, tol, &s, 1);
}

int nufft_width(int prec, double tol) { return width_of(prec, tol); }

// Every (N1, B, M) this build has pass-1 and pass-2 kernels for at a band
// count, the default schedule first (the autotuner's candidates).  Mirrors
// the feasibility rules of build_plan.
int nufft_schedules(int64_t I, int prec, double tol, std::vector<NuSchedule>& out) {
    out.clear();
    const int w = width_of(prec, tol);
    int64_t nf = 64;
    while (nf < 2 * I) nf *= 2;
    while (nf < 4 * w) nf *= 2;
    const int cs = prec == M2N_FP32 ? 8 : 16;
    if (nf <= (prec == M2N_FP32 ? 8192 : 4096)) {
        out.push_back(NuSchedule());   // single workgroup: nothing to choose
        return M2N_OK;
    }
    const int L = ilog2i(nf);
    const int p1f[][2] = {{64, 32}, {128, 32}, {256, 16}, {512, 8}, {1024, 8}, {256, 8}, {512, 16}};
    const int p1d[][2] = {{64, 32}, {128, 16}, {256, 8}, {512, 4}, {1024, 4}, {256, 4}, {512, 8}};
    // pass-2 kernels: (N2, M, KC)
    const int p2f[][3] = {{128, 1, 8}, {128, 2, 8}, {128, 4, 8}, {256, 1, 8}, {256, 2, 8}, {256, 4, 8},
                          {512, 1, 8}, {512, 2, 8}, {512, 4, 8}, {1024, 1, 8}, {1024, 2, 8},
                          {2048, 1, 8}, {4096, 1, 2}};
    const int p2d[][3] = {{128, 1, 8}, {128, 2, 8}, {128, 4, 8}, {256, 1, 8}, {256, 2, 8}, {256, 4, 8},
                          {512, 1, 8}, {512, 2, 8}, {1024, 1, 8}, {2048, 1, 2}, {4096, 1, 1}};
    int l1d = L / 2;
    if (l1d > 10) l1d = 10;
    std::vector<NuSchedule> cand;
    for (int l1 : {l1d, l1d - 1, l1d + 1}) {
        if (l1 < 6 || l1 > 10) continue;
        const int N1 = 1 << l1, N2 = (int)(nf >> l1);
        if (N2 < 128 || N2 > 4096) continue;
        int rows_max = 1;
        while (2 * rows_max * (N2 + 1) * cs + N2 * cs <= 160000) rows_max *= 2;
        const int KC = rows_max < 8 ? rows_max : 8;
        for (int bi = 0; bi < 7; ++bi) {
            const int n1b = prec == M2N_FP32 ? p1f[bi][0] : p1d[bi][0];
            const int B = prec == M2N_FP32 ? p1f[bi][1] : p1d[bi][1];
            if (n1b != N1) continue;
            const int lookback = (w - 1 + B - 1) / B;
            if (lookback >= N2 / B || N2 / B > MAX_BINS || lookback + 1 > MAXSEG) continue;
            const int n2k = prec == M2N_FP32 ? 13 : 11;
            for (int mi = 0; mi < n2k; ++mi) {
                const int* e = prec == M2N_FP32 ? p2f[mi] : p2d[mi];
                if (e[0] != N2 || e[2] != KC) continue;
                NuSchedule sc;
                sc.l1 = l1;
                sc.B = B;
                sc.M = e[1];
                cand.push_back(sc);
            }
        }
    }
    out.push_back(NuSchedule());   // the default: build_plan's own choices
    out.insert(out.end(), cand.begin(), cand.end());
    return M2N_OK;
}

void nufft_drop_plan(Ctx* ctx, int64_t I, int prec, double tol) {
    auto it = ctx->plans.find(std::make_tuple(I, prec, width_of(prec, tol)));
    if (it == ctx->plans.end()) return;
    (void)hipDeviceSynchronize();
    ctx->release(it->second->tw_fft);
    ctx->release(it->second->inv_phihat);
    ctx->plans.erase(it);
}

}  // namespace m2n
