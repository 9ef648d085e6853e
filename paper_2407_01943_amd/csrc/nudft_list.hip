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
//
// The allocation-free variant puts those partial sums in `scratch`, a
// file-scope device array of NOALLOC_SCRATCH_BYTES that every device holds
// once for the life of the process; its device address is looked up once per
// device (noalloc_scratch_init, called by m2n_create) and only that address
// is handed to the kernels.
#include <cmath>
#include <mutex>

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

// J_k(i) = sum over the chunks in order; P_i = sum_k d_k |J_k(i)|^2 over the
// K tapers of this group (tapers k0 .. k0 + K - 1 of Ktot), added to P when
// accum (the groups after the first)
__global__ __launch_bounds__(LT) void k_nudft_reduce(const cplx<double>* __restrict__ part, int nchunk, int K,
                                                     int64_t I, const double* __restrict__ weights,
                                                     double* __restrict__ P, cplx<double>* __restrict__ J,
                                                     int k0, int Ktot, int accum) {
    const int64_t i = (int64_t)blockIdx.x * LT + threadIdx.x;
    if (i >= I) return;
    const double d0 = 1.0 / Ktot;
    double p = accum ? P[i] : 0.0;
    for (int k = 0; k < K; ++k) {
        double re = 0.0, im = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            const cplx<double> v = part[((int64_t)c * K + k) * I + i];
            re += v.x;
            im += v.y;
        }
        const double d = weights ? weights[k0 + k] : d0;
        p += d * (re * re + im * im);
        if (J) {
            cplx<double> v;
            v.x = re;
            v.y = im;
            J[(int64_t)(k0 + k) * I + i] = v;
        }
    }
    P[i] = p;
}

}  // namespace

namespace {

// samples per chunk (a multiple of LS) and chunk count, so that about 1,024
// workgroups run; at most max_chunks chunks
void chunking(int64_t N, int64_t I, int64_t max_chunks, int64_t* nchunk_out, int64_t* nc_out) {
    const int64_t bx = (I + LT - 1) / LT;
    int64_t nchunk = (1024 + bx - 1) / bx;
    if (nchunk > max_chunks) nchunk = max_chunks;
    const int64_t tiles = (N + LS - 1) / LS;
    if (nchunk > tiles) nchunk = tiles;
    if (nchunk < 1) nchunk = 1;
    const int64_t nc = (tiles + nchunk - 1) / nchunk * LS;
    *nc_out = nc;
    *nchunk_out = (N + nc - 1) / nc;
}

int check_args(const double* t, const double* x, const double* w, const double* freqs, const double* P, int64_t N,
               int K, int64_t I) {
    if (!t || !x || !w || !freqs || !P || N < 1 || K < 1 || K > 64 || I < 1) {
        set_error("bad argument (N = %lld, K = %d (<= 64), I = %lld)", (long long)N, K, (long long)I);
        return M2N_ERR_ARG;
    }
    return M2N_OK;
}

// the tapers in groups of LK, one sum and one reduction per group (the
// partial sums of a group are reduced before the next group writes them)
void launch_list(hipStream_t st, const double* t, const double* x, int64_t N, const double* w, int K,
                 const double* freqs, int64_t I, const double* weights, double* P, void* J, int64_t nchunk,
                 int64_t nc, cplx<double>* part) {
    const int64_t bx = (I + LT - 1) / LT;
    for (int k0 = 0; k0 < K; k0 += LK) {
        const int kg = K - k0 < LK ? K - k0 : LK;
        hipLaunchKernelGGL(k_nudft_list, dim3((unsigned)bx, (unsigned)nchunk), dim3(LT), 0, st, t, x,
                           w + (int64_t)k0 * N, N, kg, freqs, I, nc, part);
        hipLaunchKernelGGL(k_nudft_reduce, dim3((unsigned)bx), dim3(LT), 0, st, (const cplx<double>*)part,
                           (int)nchunk, kg, I, weights, P, (cplx<double>*)J, k0, K, k0 > 0 ? 1 : 0);
    }
}

// ------------------------------------------------ allocation-free variant
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
constexpr int MAX_DEVICES = 64;
__device__ __align__(256) cplx<double> scratch[NOALLOC_SCRATCH_BYTES / sizeof(cplx<double>)];
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

int noalloc_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("device %d out of range for the scratch table", device);
        return M2N_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return M2N_OK;
    int cur = -1;
    M2N_HIP(hipGetDevice(&cur));
    if (cur != device) {
        set_error("scratch lookup for device %d while device %d is current", device, cur);
        return M2N_ERR_ARG;
    }
    void* p = nullptr;
    M2N_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
        set_error("no device address for the scratch array");
        return M2N_ERR_HIP;
    }
    g_scratch_ptr[device] = p;
    return M2N_OK;
}

size_t noalloc_scratch_bytes() { return NOALLOC_SCRATCH_BYTES; }

int nudft_list_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N, const double* w, int K,
                   const double* freqs, int64_t I, const double* weights, double* P, void* J) {
    M2N_TRY(check_args(t, x, w, freqs, P, N, K, I));
    int64_t nchunk, nc;
    chunking(N, I, INT64_MAX, &nchunk, &nc);
    void* vp;
    const int kg = K < LK ? K : LK;
    M2N_TRY(ctx->workspace("nl_part", sizeof(cplx<double>) * (size_t)nchunk * kg * I, &vp));
    {
        M2N_PROF(ctx, st, "k_nudft_list");
        launch_list(st, t, x, N, w, K, freqs, I, weights, P, J, nchunk, nc, (cplx<double>*)vp);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

// The same sums with the partial results in the per-device scratch array: no
// allocation, no workspace growth, no timing events.  Fewer sample chunks
// when min(K, 16) I nchunk complex values would not fit (the reduction order
// is still the chunk order).
int nudft_list_run_noalloc(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N, const double* w,
                           int K, const double* freqs, int64_t I, const double* weights, double* P, void* J) {
    M2N_TRY(check_args(t, x, w, freqs, P, N, K, I));
    const int kg = K < LK ? K : LK;   // tapers per group of the sums
    const size_t per_chunk = sizeof(cplx<double>) * (size_t)kg * (size_t)I;
    if (per_chunk > NOALLOC_SCRATCH_BYTES) {
        set_error("min(K, 16) I = %lld complex partial sums exceed the %zu-byte scratch of the allocation-free call",
                  (long long)kg * (long long)I, NOALLOC_SCRATCH_BYTES);
        return M2N_ERR_ARG;
    }
    void* ptr = ctx->device >= 0 && ctx->device < MAX_DEVICES ? g_scratch_ptr[ctx->device] : nullptr;
    if (!ptr) {
        set_error("scratch array of device %d not initialised", ctx->device);
        return M2N_ERR_HIP;
    }
    int64_t nchunk, nc;
    chunking(N, I, (int64_t)(NOALLOC_SCRATCH_BYTES / per_chunk), &nchunk, &nc);
    launch_list(st, t, x, N, w, K, freqs, I, weights, P, J, nchunk, nc, (cplx<double>*)ptr);
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

}  // namespace m2n
