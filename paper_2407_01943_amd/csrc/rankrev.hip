// GPSS tapers when R(B) may be numerically singular (the GEP of Sec. 3.2
// assumes R(B) positive definite, Sec. 2.1): a rank-revealing reduction.
//
// A diagonally pivoted Cholesky of R(B) takes, one at a time, the sample
// whose remaining Schur diagonal d_i is largest (ties within 1e-12 relative
// go to the smallest index), until every remaining d_i is below
// tau * 2 f_max.  With S the samples taken, R(B)_SS is positive definite
// with pivots >= tau * 2 f_max, and the samples left out are, within that
// tolerance, linear combinations of the kept ones in the band-limited space
// of B.  The tapers are the GEP tapers of the sub-series t_S (the library's
// own dense path on t_S) and vanish on the other samples, so that
// w^T R(B) w = w_S^T R(B)_SS w_S = 2 f_w holds with the full R(B).
//
// Kernels: k_rr_integral (is R(B) a multiple of the identity: then nothing
// is left out), k_rr_pick (one workgroup: the next pivot), k_rr_col (the
// pivot's column of L from its definition
//   l_{i,j} = (R(B)_{i,p} - sum_{k<j} l_{i,k} l_{p,k}) / sqrt(d_p)
// and the update d_i -= l_{i,j}^2), k_rr_compact (the sorted index list
// and t_S), k_rr_scatter (the tapers back onto all samples).  The pivot
// steps are launches of their own; the host reads the stop flag every 16
// steps.
#include <cmath>
#include <cstring>

#include "m2n_common.hpp"

namespace m2n {

namespace {

constexpr int RR_NT = 256;

struct RrState {
    int stop;     // no sample left above the tolerance
    int p;        // pivot of the current step
    int r;        // samples taken so far
    int pad;
    double inv_sdp;   // 1 / sqrt(d_p)
    double maxrem;    // largest remaining Schur diagonal (at the end)
};

__device__ __forceinline__ double rr_sinpi(double u) {
    double r = u - 2.0 * rint(0.5 * u);
    if (r > 0.5) r = 1.0 - r;
    else if (r < -0.5) r = -1.0 - r;
    return sinpi(r);
}

__device__ __forceinline__ double rr_sinc(double f, double tau) {
    if (tau == 0.0) return 2.0 * f;
    return rr_sinpi(2.0 * f * tau) / (M_PI * tau);
}

// flag[0] = 1 when every t_n is an integer (one workgroup)
__global__ __launch_bounds__(1024) void k_rr_integral(const double* __restrict__ t, int64_t N, int* flag) {
    __shared__ int ok;
    if (threadIdx.x == 0) ok = 1;
    __syncthreads();
    int mine = 1;
    for (int64_t n = threadIdx.x; n < N; n += 1024) {
        const double v = t[n];
        if (v != rint(v) || fabs(v) > 4.0e15) mine = 0;
    }
    if (!mine) atomicAnd(&ok, 0);
    __syncthreads();
    if (threadIdx.x == 0) flag[0] = ok;
}

__global__ __launch_bounds__(RR_NT) void k_rr_init(double* __restrict__ d, int* __restrict__ sel, int64_t N,
                                                   double dmax, RrState* st) {
    const int64_t i = (int64_t)blockIdx.x * RR_NT + threadIdx.x;
    if (i < N) {
        d[i] = dmax;
        sel[i] = 0;
    }
    if (i == 0) {
        st->stop = 0;
        st->p = -1;
        st->r = 0;
        st->pad = 0;
        st->inv_sdp = 0.0;
        st->maxrem = 0.0;
    }
}

// the next pivot (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void k_rr_pick(const double* __restrict__ d, int* __restrict__ sel, int64_t N,
                                                  double floor_d, int j, RrState* st) {
    __shared__ double smx[1024];
    __shared__ long long sidx[1024];
    if (st->stop) return;
    double mx = -1.0;
    for (int64_t i = threadIdx.x; i < N; i += 1024)
        if (!sel[i] && d[i] > mx) mx = d[i];
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + s]);
        __syncthreads();
    }
    mx = smx[0];
    if (!(mx >= floor_d)) {
        if (threadIdx.x == 0) {
            st->stop = 1;
            st->maxrem = mx > 0.0 ? mx : 0.0;
        }
        return;
    }
    const double thr = (1.0 - 1e-12) * mx;
    long long best = N;
    for (int64_t i = threadIdx.x; i < N; i += 1024)
        if (!sel[i] && d[i] >= thr && i < best) best = i;
    sidx[threadIdx.x] = best;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s && sidx[threadIdx.x + s] < sidx[threadIdx.x]) sidx[threadIdx.x] = sidx[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int p = (int)sidx[0];
        sel[p] = 1;
        st->p = p;
        st->r = j + 1;
        st->inv_sdp = 1.0 / sqrt(d[p]);
    }
}

// column j of L (column-major, L + j N) and the Schur diagonal update
__global__ __launch_bounds__(RR_NT) void k_rr_col(const double* __restrict__ t, int64_t N, double fmax, int j,
                                                  const RrState* st, const int* __restrict__ sel,
                                                  double* __restrict__ L, double* __restrict__ d) {
    if (st->stop) return;
    const int64_t i = (int64_t)blockIdx.x * RR_NT + threadIdx.x;
    if (i >= N) return;
    const int p = st->p;
    if (sel[i] && i != p) {
        L[(int64_t)j * N + i] = 0.0;
        return;
    }
    double v = rr_sinc(fmax, t[i] - t[p]);
    for (int k = 0; k < j; ++k) v -= L[(int64_t)k * N + i] * L[(int64_t)k * N + p];
    const double l = v * st->inv_sdp;
    L[(int64_t)j * N + i] = l;
    if (i == p) d[i] = 0.0;
    else d[i] -= l * l;
}

// the kept samples in increasing order: idx[m], pos[i] (-1 when left out),
// tS[m] = t[idx[m]] (one workgroup, chunked exclusive scan)
__global__ __launch_bounds__(1024) void k_rr_compact(const double* __restrict__ t, int64_t N,
                                                     const int* __restrict__ sel, int* __restrict__ idx,
                                                     int* __restrict__ pos, double* __restrict__ tS) {
    __shared__ int cnt[1024];
    int base = 0;
    for (int64_t c0 = 0; c0 < N; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const int s = (i < N && sel[i]) ? 1 : 0;
        cnt[threadIdx.x] = s;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int v = (int)threadIdx.x >= o ? cnt[threadIdx.x - o] : 0;
            __syncthreads();
            cnt[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < N) {
            const int m = base + cnt[threadIdx.x] - s;
            pos[i] = s ? m : -1;
            if (s) {
                idx[m] = (int)i;
                tS[m] = t[i];
            }
        }
        const int tot = cnt[1023];
        __syncthreads();
        base += tot;
    }
}

// w[k][i] = wS[k][pos[i]] on the kept samples, 0 elsewhere
__global__ __launch_bounds__(RR_NT) void k_rr_scatter(const double* __restrict__ wS, int64_t r,
                                                      const int* __restrict__ pos, int64_t N, int K,
                                                      double* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * RR_NT + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= N || k >= K) return;
    const int m = pos[i];
    w[(int64_t)k * N + i] = m >= 0 ? wS[(int64_t)k * r + m] : 0.0;
}

}  // namespace

int gep_rr(Ctx* ctx, hipStream_t st, const double* t, int64_t N, double fmax, double fw, int K, double tau,
           double* w, double* lambda, int64_t* rank) {
    if (!t || !w || !lambda || N < 1 || K < 1 || K > 64 || K > N) {
        set_error("bad argument (N = %lld, K = %d)", (long long)N, K);
        return M2N_ERR_ARG;
    }
    if (!std::isfinite(fmax) || !std::isfinite(fw) || !(fw > 0.0) || !(fw < fmax)) {
        set_error("need 0 < fw < fmax (fw = %g, fmax = %g)", fw, fmax);
        return M2N_ERR_ARG;
    }
    if (tau <= 0.0) tau = 1e-8;
    if (!(tau < 1.0)) {
        set_error("rank tolerance must be below 1 (got %g)", tau);
        return M2N_ERR_ARG;
    }
    if (N > 32768) {
        set_error("the rank-revealing reduction is limited to N <= 32768 in this build");
        return M2N_ERR_UNSUPPORTED;
    }
    const double cB = 2.0 * fmax;
    // R(B) = 2 f_max I exactly (integer t, integer 2 f_max): nothing to leave out
    M2N_TRY(ctx->pinned_erec(sizeof(RrState) + 64));
    int* hflag = (int*)ctx->erec;
    void* wflag;
    M2N_TRY(ctx->workspace("rr_flag", 64, &wflag));
    hipLaunchKernelGGL(k_rr_integral, dim3(1), dim3(1024), 0, st, t, N, (int*)wflag);
    M2N_HIP(hipMemcpyAsync(hflag, wflag, sizeof(int), hipMemcpyDeviceToHost, st));
    M2N_HIP(hipStreamSynchronize(st));
    if (*hflag && cB == std::rint(cB) && cB >= 1.0) {
        M2N_TRY(gep_run(ctx, st, t, N, fmax, fw, K, w, lambda));
        if (rank) *rank = N;
        return M2N_OK;
    }
    // workspace: L (N x N at most), d, sel, idx, pos, tS, wS, state
    const size_t al = 256;
    auto up = [&](size_t b) { return (b + al - 1) / al * al; };
    const size_t bL = up(sizeof(double) * (size_t)N * (size_t)N), bd = up(sizeof(double) * (size_t)N),
                 bi = up(sizeof(int) * (size_t)N), bw = up(sizeof(double) * (size_t)N * (size_t)K),
                 bs = up(sizeof(RrState));
    void* wsp;
    M2N_TRY(ctx->workspace("rr_work", bL + 2 * bd + 3 * bi + bw + bs, &wsp));
    char* c = (char*)wsp;
    double* L = (double*)c;
    c += bL;
    double* d = (double*)c;
    c += bd;
    double* tS = (double*)c;
    c += bd;
    int* sel = (int*)c;
    c += bi;
    int* idx = (int*)c;
    c += bi;
    int* pos = (int*)c;
    c += bi;
    double* wS = (double*)c;
    c += bw;
    RrState* dst = (RrState*)c;
    RrState* hst = (RrState*)((char*)ctx->erec + 64);
    const unsigned gN = (unsigned)((N + RR_NT - 1) / RR_NT);
    {
        M2N_PROF(ctx, st, "k_rr_init");
        hipLaunchKernelGGL(k_rr_init, dim3(gN), dim3(RR_NT), 0, st, d, sel, N, cB, dst);
    }
    const double floor_d = tau * cB;
    for (int64_t j = 0; j < N; ++j) {
        {
            M2N_PROF(ctx, st, "k_rr_pick");
            hipLaunchKernelGGL(k_rr_pick, dim3(1), dim3(1024), 0, st, (const double*)d, sel, N, floor_d, (int)j,
                               dst);
        }
        {
            M2N_PROF(ctx, st, "k_rr_col");
            hipLaunchKernelGGL(k_rr_col, dim3(gN), dim3(RR_NT), 0, st, t, N, fmax, (int)j, (const RrState*)dst,
                               (const int*)sel, L, d);
        }
        if ((j & 15) == 15 || j + 1 == N) {
            M2N_HIP(hipGetLastError());
            M2N_HIP(hipMemcpyAsync(hst, dst, sizeof(RrState), hipMemcpyDeviceToHost, st));
            M2N_HIP(hipStreamSynchronize(st));
            if (hst->stop) break;
        }
    }
    M2N_HIP(hipMemcpyAsync(hst, dst, sizeof(RrState), hipMemcpyDeviceToHost, st));
    M2N_HIP(hipStreamSynchronize(st));
    const int64_t r = hst->r;
    if (rank) *rank = r;
    if (r < K) {
        set_error("numerical rank %lld of R(B) at tolerance %g is below K = %d", (long long)r, tau, K);
        return M2N_ERR_NOT_PD;
    }
    {
        M2N_PROF(ctx, st, "k_rr_compact");
        hipLaunchKernelGGL(k_rr_compact, dim3(1), dim3(1024), 0, st, t, N, (const int*)sel, idx, pos, tS);
    }
    M2N_HIP(hipGetLastError());
    // the GEP of the sub-series (its own t check and path choice)
    M2N_TRY(gep_run(ctx, st, tS, r, fmax, fw, K, wS, lambda));
    {
        M2N_PROF(ctx, st, "k_rr_scatter");
        hipLaunchKernelGGL(k_rr_scatter, dim3(gN, (unsigned)K), dim3(RR_NT), 0, st, (const double*)wS, r,
                           (const int*)pos, N, K, w);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

}  // namespace m2n
