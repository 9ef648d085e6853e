// One sub-band of the multiband partition (Sec. 2.4, Sec. 3.1-3.2): the
// eigencoefficients of complex tapers on frequencies relative to the nominal
// band centre, and their power average.
//
// With w_k = a_k + j b_k (planar: the K real parts, then the K imaginary
// parts, as gpss_tapers_subband writes them), conj(w_k) x = a_k x - j b_k x,
// so J_k = N[a_k x] - j N[b_k x] where N[.] is the type-1 NuFFT of a real
// tapered series.  The 2K real parts go through the full-band NuFFT as 2K
// tapers; k_sb_combine forms J_k and P_i = sum_k d_k |J_k(i)|^2.
#include <cmath>
#include <string>
#include <thread>

#include "m2n_common.hpp"

namespace m2n {

// J_k(i) = Jp[k][i] - j Jp[K + k][i];  P[i] = sum_k d_k |J_k(i)|^2 with
// d_k = weights[k] or 1/K.  One band per thread; J may be null.
template <typename R>
__global__ __launch_bounds__(256) void k_sb_combine(const cplx<R>* __restrict__ Jp, int K, int64_t I,
                                                    const double* __restrict__ weights,
                                                    R* __restrict__ P, cplx<R>* __restrict__ J) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= I) return;
    const R d0 = (R)(1.0 / K);
    R p = 0;
    for (int k = 0; k < K; ++k) {
        const cplx<R> a = Jp[(int64_t)k * I + i], b = Jp[(int64_t)(K + k) * I + i];
        cplx<R> j;
        j.x = a.x + b.y;
        j.y = a.y - b.x;
        const R d = weights ? (R)weights[k] : d0;
        p += d * (j.x * j.x + j.y * j.y);
        if (J) J[(int64_t)k * I + i] = j;
    }
    P[i] = p;
}

int subband_psd_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N,
                    const double* w, int K, double f_lo, double df, int64_t I, int prec, double tol,
                    const double* weights, void* P, void* J) {
    if (K < 1 || 2 * K > 64 || I < 1) {
        set_error("need 1 <= K <= 32 and I >= 1 (K = %d, I = %lld)", K, (long long)I);
        return M2N_ERR_ARG;
    }
    if (prec != M2N_FP32 && prec != M2N_FP64) {
        set_error("prec must be M2N_FP32 or M2N_FP64");
        return M2N_ERR_ARG;
    }
    const size_t cs = prec == M2N_FP32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    void* vJ;
    M2N_TRY(ctx->workspace("sb_J", cs * 2 * (size_t)K * (size_t)I, &vJ));
    M2N_TRY(nufft_run(ctx, st, t, x, N, w, 2 * K, f_lo, df, I, prec, tol, nullptr, nullptr, 0.0, 0.0,
                      nullptr, nullptr, vJ, nullptr));
    const dim3 g((unsigned)((I + 255) / 256));
    M2N_PROF(ctx, st, "k_sb_combine");
    if (prec == M2N_FP32)
        hipLaunchKernelGGL(k_sb_combine<float>, g, dim3(256), 0, st, (const cplx<float>*)vJ, K, I, weights,
                           (float*)P, (cplx<float>*)J);
    else
        hipLaunchKernelGGL(k_sb_combine<double>, g, dim3(256), 0, st, (const cplx<double>*)vJ, K, I, weights,
                           (double*)P, (cplx<double>*)J);
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

// Q sub-bands at once (Sec. 3.1: the sub-bands are independent).  Each runs
// gpss_tapers_subband's path on a child context of its own (workspace, aux
// stream, pinned records) and a stream of its own, from a host thread of its
// own: one dense factorisation leaves most compute units idle, so the panel
// chains of different sub-bands overlap.  The child streams first wait for
// the caller's stream (t may still be in flight there); the call returns once
// every sub-band is complete.  The first failing sub-band's error is
// reported with its index.
int multiband_run(Ctx* ctx, hipStream_t st, const double* t, int64_t N, double fw, int K, const m2n_subband* sb,
                  int Q) {
    while ((int)ctx->subs.size() < Q) {
        m2n_ctx* c = nullptr;
        M2N_TRY(m2n_create(ctx->device, ctx->budget, &c));
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            m2n_destroy(c);
            set_error("hipStreamCreateWithFlags failed");
            return M2N_ERR_HIP;
        }
        ctx->subs.push_back(c);
        ctx->sub_streams.push_back(s);
    }
    M2N_HIP(hipSetDevice(ctx->device));
    hipEvent_t ready = nullptr;
    M2N_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    if (hipEventRecord(ready, st) != hipSuccess) {
        (void)hipEventDestroy(ready);
        set_error("hipEventRecord failed");
        return M2N_ERR_HIP;
    }
    std::vector<int> rc((size_t)Q, M2N_OK);
    std::vector<std::string> msg((size_t)Q);
    std::vector<std::thread> th;
    th.reserve((size_t)Q);
    for (int q = 0; q < Q; ++q) {
        th.emplace_back([&, q]() {
            if (hipSetDevice(ctx->device) != hipSuccess ||
                hipStreamWaitEvent(ctx->sub_streams[q], ready, 0) != hipSuccess) {
                rc[q] = M2N_ERR_HIP;
                msg[q] = "stream setup failed";
                return;
            }
            rc[q] = gep_subband(ctx->subs[q], ctx->sub_streams[q], t, N, sb[q].fmin, sb[q].fmax, fw, sb[q].fc0,
                                K, sb[q].w, sb[q].lambda);
            if (rc[q] != M2N_OK) msg[q] = m2n_last_error(nullptr);   // the worker's own error text
        });
    }
    for (auto& x : th) x.join();
    (void)hipEventDestroy(ready);
    for (int q = 0; q < Q; ++q)
        if (rc[q] != M2N_OK) {
            set_error("sub-band %d: %s", q, msg[q].c_str());
            return rc[q];
        }
    return M2N_OK;
}

}  // namespace m2n
