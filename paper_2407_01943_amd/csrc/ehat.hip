// Suboptimality estimate for any sampling times (Sec. 3.5 measure, Appendix B
// Rayleigh quotient of the shifted tapers):
//
//   Ehat_i = (1/K) sum_k |lambda_k - 2 f_w lambda_k / D_k(i)|,
//   D_k(i) = (E_i w_k)^* R(B) (E_i w_k).
//
// Writing R(B) as the integral of e^{j 2 pi f (t_n - t_m)} over |f| <= f_max
// turns the quadratic form into an integral of the taper's spectral window,
//
//   D_k(i) = int_{Df_i - f_max}^{Df_i + f_max} |W_k(f)|^2 df,
//   W_k(f) = sum_n w_k(t_n) e^{-j 2 pi f t_n},  Df_i = f_lo + i df,
//
// (W_k is real-tapered, so |W_k(-f)| = |W_k(f)|).  The windows of consecutive
// bands are shifted by df, so with M = floor(2 f_max / df) and r the fraction
// left over,
//
//   D_k(i) = sum_{j=i}^{i+M-1} C_k(j) + C'_k(i),
//   C_k(j)  = int over [c_j, c_j + df]          of |W_k|^2,  c_j = f_lo - f_max + j df,
//   C'_k(i) = int over [c_{i+M}, c_{i+M} + r df] of |W_k|^2.
//
// Each cell integral is a Gauss-Legendre sum; the nodes of one order q sit at
// the same offset in every cell, so the values |W_k|^2 at them are one type-1
// NuFFT of the bare tapers (x = 1) on an arithmetic progression of band
// centres: the library's own NuFFT, batched over (node, taper) pairs with one
// taper per series, so that its P output is |W_k|^2 itself.  |W_k|^2 is a sum
// of exponentials e^{-j 2 pi f tau} with |tau| <= t_N - t_1, so the order is
// chosen for the largest such exponential over one cell.  The sum over the
// window is a difference of FP64 prefix sums of the cells.  Valid for any t;
// when R(B) is a multiple of the identity the NuFFT pass writes the
// band-constant value directly and none of this runs.
#include <cmath>
#include <cstring>
#include <mutex>

#include "m2n_common.hpp"

namespace m2n {

namespace {

constexpr int EH_NT = 256;          // threads per workgroup
constexpr int EH_CELLS = 1024;      // cells per block of the prefix sum
constexpr int EH_MAXQ = 64;         // largest quadrature order

struct QuadW {
    double w[EH_MAXQ];   // Gauss-Legendre weights times half the cell width
};

__global__ __launch_bounds__(EH_NT) void k_eh_ones(double* __restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * EH_NT + threadIdx.x;
    if (i < n) v[i] = 1.0;
}

// sum over the 256 threads of a workgroup in a fixed order; thread 0 gets it
__device__ __forceinline__ double eh_block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < EH_NT / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

// C[k][j] = sum_q qw[q] |W_k(c_j + node_q)|^2 for one block of EH_CELLS cells
// (grid: blocks x K); bsum[k][b] = the block's total
template <typename R>
__global__ __launch_bounds__(EH_NT) void k_eh_cells(const R* __restrict__ pw, int nq, int K, int64_t nC, QuadW qw,
                                                     double* __restrict__ C, double* __restrict__ bsum, int nblk) {
    __shared__ double red[EH_NT / 64];
    const int k = blockIdx.y, b = blockIdx.x;
    const int64_t j0 = (int64_t)b * EH_CELLS;
    double part = 0.0;
    for (int u = threadIdx.x; u < EH_CELLS; u += EH_NT) {
        const int64_t j = j0 + u;
        if (j >= nC) break;
        double c = 0.0;
        for (int q = 0; q < nq; ++q) c += qw.w[q] * (double)pw[((int64_t)q * K + k) * nC + j];
        C[(int64_t)k * nC + j] = c;
        part += c;
    }
    const double s = eh_block_sum(part, red);
    if (threadIdx.x == 0) bsum[(int64_t)k * nblk + b] = s;
}

// exclusive prefix of the block totals of taper k = blockIdx.x, in block
// order: base[k][b] for b = 0..nblk (base[k][nblk] = the total)
__global__ __launch_bounds__(64) void k_eh_scan(const double* __restrict__ bsum, int nblk,
                                                double* __restrict__ base) {
    if (threadIdx.x != 0) return;
    const int k = blockIdx.x;
    double run = 0.0;
    for (int b = 0; b < nblk; ++b) {
        base[(int64_t)k * (nblk + 1) + b] = run;
        run += bsum[(int64_t)k * nblk + b];
    }
    base[(int64_t)k * (nblk + 1) + nblk] = run;
}

// S[k][j] = sum_{j' < j} C[k][j'] for j = 0..nC: the block's base plus the
// exclusive scan inside the block (thread-serial runs of four, then the
// threads in order)
__global__ __launch_bounds__(EH_NT) void k_eh_prefix(const double* __restrict__ C, int64_t nC,
                                                     const double* __restrict__ base, int nblk,
                                                     double* __restrict__ S) {
    constexpr int PER = EH_CELLS / EH_NT;
    __shared__ double tot[EH_NT];
    const int k = blockIdx.y, b = blockIdx.x;
    const int64_t j0 = (int64_t)b * EH_CELLS + (int64_t)threadIdx.x * PER;
    double v[PER];
    double sum = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int64_t j = j0 + u;
        v[u] = j < nC ? C[(int64_t)k * nC + j] : 0.0;
        sum += v[u];
    }
    tot[threadIdx.x] = sum;
    __syncthreads();
    double run = base[(int64_t)k * (nblk + 1) + b];
    for (int i = 0; i < (int)threadIdx.x; ++i) run += tot[i];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int64_t j = j0 + u;
        if (j <= nC) S[(int64_t)k * (nC + 1) + j] = run;
        run += v[u];
    }
}

// Ehat_i from the window sums S[k][i + M] - S[k][i] and the partial cell
// (pr: |W_k|^2 at the partial cell's nodes, nqr orders, or none)
template <typename R>
__global__ __launch_bounds__(EH_NT) void k_eh_final(const double* __restrict__ S, int64_t nC, int64_t M,
                                                     const R* __restrict__ pr, int nqr, QuadW qwr, int K,
                                                     const double* __restrict__ lambda, double fw, int64_t I,
                                                     R* __restrict__ E) {
    const int64_t i = (int64_t)blockIdx.x * EH_NT + threadIdx.x;
    if (i >= I) return;
    double e = 0.0;
    for (int k = 0; k < K; ++k) {
        double D = 0.0;
        if (M > 0) D = S[(int64_t)k * (nC + 1) + i + M] - S[(int64_t)k * (nC + 1) + i];
        for (int q = 0; q < nqr; ++q) D += qwr.w[q] * (double)pr[((int64_t)q * K + k) * I + i];
        const double lam = lambda[k];
        e += fabs(lam - 2.0 * fw * lam / D);
    }
    E[i] = (R)(e / (double)K);
}

// ------------------------------------------------------------ host side
std::mutex g_gl_mu;
std::map<int, std::pair<std::vector<double>, std::vector<double>>> g_gl;   // order -> nodes, weights
std::map<long long, int> g_order;                                           // ceil(16 beta) -> order

void gl_rule(int p, std::vector<double>& x, std::vector<double>& w) {
    std::lock_guard<std::mutex> lk(g_gl_mu);
    auto it = g_gl.find(p);
    if (it == g_gl.end()) {
        std::vector<double> gx, gw;
        gauss_legendre(p, gx, gw);
        it = g_gl.emplace(p, std::make_pair(gx, gw)).first;
    }
    x = it->second.first;
    w = it->second.second;
}

// the smallest Gauss-Legendre order (plus a margin of two) whose rule on
// [-1, 1] integrates e^{j b x} to within 1e-15 of 2 sin(b)/b for every
// 0 <= b <= beta; -1 if none up to EH_MAXQ
int gl_order_for(double beta) {
    const long long key = (long long)std::ceil(beta * 16.0);
    const double bq = (double)key / 16.0;   // rounded up: a conservative order
    {
        std::lock_guard<std::mutex> lk(g_gl_mu);
        auto it = g_order.find(key);
        if (it != g_order.end()) return it->second;
    }
    int found = -1;
    for (int p = 2; p <= EH_MAXQ - 2; ++p) {
        std::vector<double> x, w;
        gl_rule(p, x, w);
        double err = 0.0;
        for (int s = 0; s <= 64; ++s) {
            const double b = bq * s / 64.0;
            double q = 0.0;
            for (int i = 0; i < p; ++i) q += w[i] * std::cos(b * x[i]);
            const double ex = b == 0.0 ? 2.0 : 2.0 * std::sin(b) / b;
            err = std::max(err, std::fabs(q - ex));
        }
        if (err <= 1e-15) {
            found = p + 2;
            break;
        }
    }
    std::lock_guard<std::mutex> lk(g_gl_mu);
    g_order[key] = found;
    return found;
}

// |W_k|^2 at the nodes f_first + j df + off_q, j < nb, for every node q and
// taper k, into pw[(q K + k) nb + j] (type R): one batched NuFFT launch set
int window_samples(Ctx* ctx, hipStream_t st, const NuSeriesIn& s, const double* ones, double f_first, double df,
                   int64_t nb, const std::vector<double>& off, int prec, double tol, void* pw) {
    const int K = s.K;
    const size_t rb = prec == M2N_FP32 ? sizeof(float) : sizeof(double);
    std::vector<NuSeriesIn> ser;
    ser.reserve(off.size() * (size_t)K);
    for (size_t q = 0; q < off.size(); ++q) {
        for (int k = 0; k < K; ++k) {
            NuSeriesIn n;
            n.t = s.t;
            n.x = ones;
            n.w = s.w + (int64_t)k * s.N;
            n.N = s.N;
            n.K = 1;
            n.f_lo = f_first + off[q];
            n.df = df;
            n.P = (char*)pw + ((q * (size_t)K + (size_t)k) * (size_t)nb) * rb;
            ser.push_back(n);
        }
    }
    return nufft_run_batch(ctx, st, nb, prec, tol, ser.data(), (int)ser.size());
}

template <typename R>
int ehat_typed(Ctx* ctx, hipStream_t st, int64_t I, int prec, double tol, const NuSeriesIn& s, double span) {
    const int K = s.K;
    const double df = s.df, fmax = s.fmax;
    // window = M whole cells plus a fraction r of one
    const double ratio = 2.0 * fmax / df;
    if (!(ratio < 1e15)) {
        set_error("Ehat: 2 f_max / df = %g is too large", ratio);
        return M2N_ERR_UNSUPPORTED;
    }
    int64_t M = (int64_t)std::floor(ratio);
    double r = ratio - (double)M;
    if (r < 1e-13 * std::max(1.0, ratio)) r = 0.0;
    if (1.0 - r < 1e-13 * std::max(1.0, ratio)) {
        M += 1;
        r = 0.0;
    }
    const int64_t nC = M > 0 ? I + M - 1 : 0;
    if (nC > (int64_t(1) << 21)) {
        set_error("Ehat with a non-diagonal R(B) needs I + 2 f_max / df <= 2^21 + 1 (I = %lld, 2 f_max / df = %g)",
                  (long long)I, ratio);
        return M2N_ERR_UNSUPPORTED;
    }
    // quadrature orders for a whole cell and for the partial one
    const double beta = M_PI * df * span;
    const int p = nC > 0 ? gl_order_for(beta) : 0;
    const int pr = r > 0.0 ? gl_order_for(beta * r) : 0;
    if (p < 0 || pr < 0) {
        set_error("Ehat: band spacing too coarse for the window quadrature (df (t_N - t_1) = %g)", df * span);
        return M2N_ERR_UNSUPPORTED;
    }
    const size_t rb = sizeof(R);
    const int64_t nblk = (nC + EH_CELLS) / EH_CELLS;   // covers j = 0..nC
    // workspace: ones [N], |W|^2 samples, cells, block totals and bases, prefix
    size_t off_pw = 0;
    size_t bytes = ((size_t)s.N * 8 + 255) & ~size_t(255);
    off_pw = bytes;
    bytes += (((size_t)p * K * (size_t)nC + (size_t)pr * K * (size_t)I) * rb + 255) & ~size_t(255);
    const size_t off_c = bytes;
    bytes += ((size_t)K * (size_t)nC * 8 + 255) & ~size_t(255);
    const size_t off_bs = bytes;
    bytes += ((size_t)K * (size_t)nblk * 8 + 255) & ~size_t(255);
    const size_t off_base = bytes;
    bytes += ((size_t)K * (size_t)(nblk + 1) * 8 + 255) & ~size_t(255);
    const size_t off_s = bytes;
    bytes += ((size_t)K * (size_t)(nC + 1) * 8 + 255) & ~size_t(255);
    void* wsp;
    M2N_TRY(ctx->workspace("eh_work", bytes, &wsp));
    char* base = (char*)wsp;
    double* ones = (double*)base;
    R* pw = (R*)(base + off_pw);
    R* pwr = pw + (size_t)p * K * (size_t)nC;
    double* C = (double*)(base + off_c);
    double* bsum = (double*)(base + off_bs);
    double* bbase = (double*)(base + off_base);
    double* S = (double*)(base + off_s);
    {
        M2N_PROF(ctx, st, "k_eh_ones");
        hipLaunchKernelGGL(k_eh_ones, dim3((unsigned)((s.N + EH_NT - 1) / EH_NT)), dim3(EH_NT), 0, st, ones, s.N);
    }
    M2N_HIP(hipGetLastError());
    QuadW qw{}, qwr{};
    if (p > 0) {
        std::vector<double> x, w, off((size_t)p);
        gl_rule(p, x, w);
        for (int q = 0; q < p; ++q) {
            off[q] = 0.5 * df * (1.0 + x[q]);
            qw.w[q] = 0.5 * df * w[q];
        }
        M2N_TRY(window_samples(ctx, st, s, ones, s.f_lo - fmax, df, nC, off, prec, tol, pw));
        {
            M2N_PROF(ctx, st, "k_eh_cells");
            hipLaunchKernelGGL((k_eh_cells<R>), dim3((unsigned)nblk, (unsigned)K), dim3(EH_NT), 0, st,
                               (const R*)pw, p, K, nC, qw, C, bsum, (int)nblk);
        }
        {
            M2N_PROF(ctx, st, "k_eh_scan");
            hipLaunchKernelGGL(k_eh_scan, dim3((unsigned)K), dim3(64), 0, st, (const double*)bsum, (int)nblk,
                               bbase);
        }
        {
            M2N_PROF(ctx, st, "k_eh_prefix");
            hipLaunchKernelGGL(k_eh_prefix, dim3((unsigned)nblk, (unsigned)K), dim3(EH_NT), 0, st,
                               (const double*)C, nC, (const double*)bbase, (int)nblk, S);
        }
        M2N_HIP(hipGetLastError());
    }
    if (pr > 0) {
        std::vector<double> x, w, off((size_t)pr);
        gl_rule(pr, x, w);
        for (int q = 0; q < pr; ++q) {
            off[q] = 0.5 * r * df * (1.0 + x[q]);
            qwr.w[q] = 0.5 * r * df * w[q];
        }
        M2N_TRY(window_samples(ctx, st, s, ones, s.f_lo - fmax + (double)M * df, df, I, off, prec, tol, pwr));
    }
    {
        M2N_PROF(ctx, st, "k_eh_final");
        hipLaunchKernelGGL((k_eh_final<R>), dim3((unsigned)((I + EH_NT - 1) / EH_NT)), dim3(EH_NT), 0, st,
                           (const double*)S, nC, M, (const R*)pwr, pr, qwr, K, s.lambda, s.fw, I, (R*)s.E);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

}  // namespace

int ehat_general(Ctx* ctx, hipStream_t st, int64_t I, int prec, double tol, const NuSeriesIn& s, double span) {
    if (prec == M2N_FP32) return ehat_typed<float>(ctx, st, I, prec, tol, s, span);
    return ehat_typed<double>(ctx, st, I, prec, tol, s, span);
}

}  // namespace m2n
