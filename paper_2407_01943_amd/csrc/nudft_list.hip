// Eigencoefficients at an arbitrary list of band centres (Sec. 3.2: the band
// centres of an analysis need not form an arithmetic progression), by direct
// FP64 summation on the GPU:
//   J_k(i) = sum_n w_k(t_n) x(t_n) e^{-j 2 pi f_i t_n},  P_i = sum_k d_k |J_k(i)|^2.
// The cost is N I complex exponentials, the right tool for a modest number of
// centres; for many equally spaced centres the type-1 NuFFT path is O(N log N).
// Each thread owns one centre and one chunk of the samples (grid y), so that
// few centres still fill the GPU; a workgroup stages a tile of samples (t_n and
// the K tapered samples) in LDS; the phase f_i t_n is split into an exact
// product and its rounding error (FMA) and reduced modulo 1 before sincospi.
// The chunks' partial sums go to a workspace and k_nudft_reduce adds them in
// chunk order (deterministic) and forms J and P.
#include <cmath>

#include "m2n_common.hpp"

namespace m2n {

namespace {

constexpr int LT = 256;       // threads (centres) per workgroup
constexpr int LS = 128;       // samples per LDS tile
constexpr int LK = 16;        // tapers per call

// part[((c K + k) I + i)] = partial J_k(i) of sample chunk c = blockIdx.y
__global__ __launch_bounds__(LT) void k_nudft_list(const double* __restrict__ t, const double* __restrict__ x,
                                                   const double* __restrict__ w, int64_t N, int K,
                                                   const double* __restrict__ freqs, int64_t I, int64_t nc,
                                                   cplx<double>* __restrict__ part) {
    __shared__ double ts[LS];
    __shared__ double ys[LK][LS];
    const int64_t i = (int64_t)blockIdx.x * LT + threadIdx.x;
    const double f = i < I ? freqs[i] : 0.0;
    double re[LK], im[LK];
#pragma unroll
    for (int k = 0; k < LK; ++k) {
        re[k] = 0.0;
        im[k] = 0.0;
    }
    const int64_t c0 = (int64_t)blockIdx.y * nc, c1 = c0 + nc < N ? c0 + nc : N;
    for (int64_t n0 = c0; n0 < c1; n0 += LS) {
        const int cnt = (int)(c1 - n0 < LS ? c1 - n0 : LS);
        __syncthreads();
        for (int e = threadIdx.x; e < LS; e += LT) ts[e] = e < cnt ? t[n0 + e] : 0.0;
        for (int e = threadIdx.x; e < LK * LS; e += LT) {
            const int k = e / LS, j = e % LS;
            ys[k][j] = (j < cnt && k < K) ? w[(int64_t)k * N + n0 + j] * x[n0 + j] : 0.0;
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const double hi = f * ts[j];
            const double lo = fma(f, ts[j], -hi);
            const double r = (hi - rint(hi)) + lo;
            double sn, cs;
            sincospi(2.0 * r, &sn, &cs);
#pragma unroll
            for (int k = 0; k < LK; ++k) {
                re[k] += ys[k][j] * cs;
                im[k] -= ys[k][j] * sn;
            }
        }
    }
    if (i >= I) return;
#pragma unroll
    for (int k = 0; k < LK; ++k) {
        if (k >= K) break;
        cplx<double> v;
        v.x = re[k];
        v.y = im[k];
        part[((int64_t)blockIdx.y * K + k) * I + i] = v;
    }
}

// J_k(i) = sum over the chunks in order; P_i = sum_k d_k |J_k(i)|^2
__global__ __launch_bounds__(LT) void k_nudft_reduce(const cplx<double>* __restrict__ part, int nchunk, int K,
                                                     int64_t I, const double* __restrict__ weights,
                                                     double* __restrict__ P, cplx<double>* __restrict__ J) {
    const int64_t i = (int64_t)blockIdx.x * LT + threadIdx.x;
    if (i >= I) return;
    const double d0 = 1.0 / K;
    double p = 0.0;
    for (int k = 0; k < K; ++k) {
        double re = 0.0, im = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            const cplx<double> v = part[((int64_t)c * K + k) * I + i];
            re += v.x;
            im += v.y;
        }
        const double d = weights ? weights[k] : d0;
        p += d * (re * re + im * im);
        if (J) {
            cplx<double> v;
            v.x = re;
            v.y = im;
            J[(int64_t)k * I + i] = v;
        }
    }
    P[i] = p;
}

}  // namespace

int nudft_list_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N, const double* w, int K,
                   const double* freqs, int64_t I, const double* weights, double* P, void* J) {
    if (!t || !x || !w || !freqs || !P || N < 1 || K < 1 || K > LK || I < 1) {
        set_error("bad argument (N = %lld, K = %d (<= %d), I = %lld)", (long long)N, K, LK, (long long)I);
        return M2N_ERR_ARG;
    }
    // sample chunks of a multiple of LS so that about 1,024 workgroups run
    const int64_t bx = (I + LT - 1) / LT;
    int64_t nchunk = (1024 + bx - 1) / bx;
    const int64_t tiles = (N + LS - 1) / LS;
    if (nchunk > tiles) nchunk = tiles;
    const int64_t nc = (tiles + nchunk - 1) / nchunk * LS;
    nchunk = (N + nc - 1) / nc;
    void* vp;
    M2N_TRY(ctx->workspace("nl_part", sizeof(cplx<double>) * (size_t)nchunk * K * I, &vp));
    {
        M2N_PROF(ctx, st, "k_nudft_list");
        hipLaunchKernelGGL(k_nudft_list, dim3((unsigned)bx, (unsigned)nchunk), dim3(LT), 0, st, t, x, w, N, K, freqs,
                           I, nc, (cplx<double>*)vp);
    }
    {
        M2N_PROF(ctx, st, "k_nudft_reduce");
        hipLaunchKernelGGL(k_nudft_reduce, dim3((unsigned)bx), dim3(LT), 0, st, (const cplx<double>*)vp, (int)nchunk,
                           K, I, weights, P, (cplx<double>*)J);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

}  // namespace m2n
