// Eigencoefficients and P at an arbitrary list of band centres by a type-3
// NuFFT (Sec. 3.2: the centres of the analysis bands need not be equally
// spaced):
//   J_k(f_i) = sum_n w_k(t_n) x(t_n) e^{-j 2 pi f_i t_n},  P_i = sum_k d_k |J_k(f_i)|^2.
//
// With t_c a centre of the sampling span (an integer, so that t_n - t_c is
// exact) and ~t_n = t_n - t_c, |~t_n| <= X:
//   J_k(f) = e^{-j 2 pi f t_c} sum_n c_nk e^{-j 2 pi f ~t_n},  c_nk = w_k(t_n) x(t_n).
// Let psi(f) = phi(2 f / (w d)) be the exponential-of-semicircle kernel over
// w cells of a frequency grid f_m = f_0 + m d, and Psi(tau) = int psi(f)
// e^{j 2 pi f tau} df its Fourier transform.  By Poisson summation
//   d sum_m psi(f - f_m) e^{-j 2 pi f_m tau} = sum_p Psi(tau - p/d) e^{-j 2 pi f (tau - p/d)},
// and with d = 1/(4 X) (twice oversampled over the span) every alias p != 0
// sits at |tau - p/d| >= 3X, where Psi has decayed to the kernel's tolerance.
// So, with the samples pre-divided by Psi,
//   G_k(f_m) = sum_n (c_nk / Psi(~t_n)) e^{-j 2 pi f_m ~t_n}       (a type-1 NuFFT on
//                                                                    the uniform grid f_m)
//   J_k(f_i) = e^{-j 2 pi f_i t_c} d sum_m G_k(f_m) psi(f_i - f_m)   (w grid values per
//                                                                    target)
// The first step is the library's own type-1 NuFFT (the division by Psi is
// folded into x); the second is k_t3_interp.  Cost: one type-1 NuFFT of
// about 4 X (f_max - f_min) bands plus w K complex products per target,
// whatever the number of targets.
#include <cmath>
#include <cstring>

#include "m2n_common.hpp"

namespace m2n {

namespace {

constexpr int T3_NT = 256;

__device__ __forceinline__ double t3_phi(double z, double beta) {
    const double a = 1.0 - z * z;
    return a > 0.0 ? exp(beta * (sqrt(a) - 1.0)) : 0.0;
}

// min and max of t and of the targets (one workgroup): rec[0..3]
__global__ __launch_bounds__(1024) void k_t3_range(const double* __restrict__ t, int64_t N,
                                                   const double* __restrict__ f, int64_t I, double* rec) {
    __shared__ double red[4][1024];
    double a = INFINITY, b = -INFINITY, c = INFINITY, d = -INFINITY;
    for (int64_t n = threadIdx.x; n < N; n += 1024) {
        a = fmin(a, t[n]);
        b = fmax(b, t[n]);
    }
    for (int64_t i = threadIdx.x; i < I; i += 1024) {
        c = fmin(c, f[i]);
        d = fmax(d, f[i]);
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    red[2][threadIdx.x] = c;
    red[3][threadIdx.x] = d;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
            red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + s]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rec[0] = red[0][0];
        rec[1] = red[1][0];
        rec[2] = red[2][0];
        rec[3] = red[3][0];
        __threadfence_system();
    }
}

constexpr int T3_MAXQ = 64;
struct T3Quad {
    double z[T3_MAXQ], wq[T3_MAXQ];   // the positive Gauss-Legendre nodes of [-1, 1] and their weights
    int nq;
};

// ~t_n = t_n - t_c and x'_n = x_n / Psi(~t_n),
//   Psi(tau) = (w d / 2) int_{-1}^{1} phi(z) cos(pi w d tau z) dz
__global__ __launch_bounds__(T3_NT) void k_t3_prep(const double* __restrict__ t, const double* __restrict__ x,
                                                   int64_t N, double tc, double wd, double beta, T3Quad q,
                                                   double* __restrict__ tt, double* __restrict__ xx) {
    const int64_t n = (int64_t)blockIdx.x * T3_NT + threadIdx.x;
    if (n >= N) return;
    const double tau = t[n] - tc;
    double s = 0.0;
    for (int j = 0; j < q.nq; ++j) s += q.wq[j] * t3_phi(q.z[j], beta) * cospi(wd * tau * q.z[j]);
    const double Psi = wd * s;   // (w d / 2) * 2 * int_0^1
    tt[n] = tau;
    xx[n] = x[n] / Psi;
}

// J_k(f_i) = e^{-j 2 pi f_i t_c} d sum_r G_k(f_{m0 + r}) psi(f_i - f_{m0 + r}), P_i
template <typename R>
__global__ __launch_bounds__(T3_NT) void k_t3_interp(const cplx<R>* __restrict__ G, int64_t M, int K,
                                                     const double* __restrict__ f, int64_t I, double f0, double d,
                                                     int w, double beta, double tc,
                                                     const double* __restrict__ weights, R* __restrict__ P,
                                                     cplx<R>* __restrict__ J) {
    const int64_t i = (int64_t)blockIdx.x * T3_NT + threadIdx.x;
    if (i >= I) return;
    const double fi = f[i];
    const double u = (fi - f0) / d;                       // grid coordinate of the target
    const int64_t m0 = (int64_t)ceil(u - 0.5 * (double)w);
    double ker[32];
    for (int r = 0; r < w; ++r) ker[r] = d * t3_phi(2.0 * (u - (double)(m0 + r)) / (double)w, beta);
    // e^{-j 2 pi f_i t_c}: the exact product split, reduced modulo 1
    const double ph = fi * tc, pl = fma(fi, tc, -ph);
    double sn, cs;
    sincospi(2.0 * ((ph - rint(ph)) + pl), &sn, &cs);
    double p = 0.0;
    for (int k = 0; k < K; ++k) {
        const cplx<R>* g = G + (int64_t)k * M + m0;
        double re = 0.0, im = 0.0;
        for (int r = 0; r < w; ++r) {
            re += ker[r] * (double)g[r].x;
            im += ker[r] * (double)g[r].y;
        }
        // (re + j im) (cs - j sn)
        const double jr = re * cs + im * sn, ji = im * cs - re * sn;
        const double dk = weights ? weights[k] : 1.0 / K;
        p += dk * (jr * jr + ji * ji);
        if (J) J[(int64_t)k * I + i] = {(R)jr, (R)ji};
    }
    P[i] = (R)p;
}

}  // namespace

int nufft3_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N, const double* w, int K,
               const double* freqs, int64_t I, int prec, double tol, const double* weights, void* P, void* J) {
    if (!t || !x || !w || !freqs || !P || N < 1 || K < 1 || K > 64 || I < 1) {
        set_error("bad argument (N = %lld, K = %d, I = %lld)", (long long)N, K, (long long)I);
        return M2N_ERR_ARG;
    }
    if (prec != M2N_FP32 && prec != M2N_FP64) {
        set_error("prec must be M2N_FP32 or M2N_FP64");
        return M2N_ERR_ARG;
    }
    // the span of t and of the targets (one host round trip)
    M2N_TRY(ctx->pinned_erec(4 * sizeof(double)));
    double* rec = (double*)ctx->erec;
    {
        M2N_PROF(ctx, st, "k_t3_range");
        hipLaunchKernelGGL(k_t3_range, dim3(1), dim3(1024), 0, st, t, N, freqs, I, rec);
    }
    M2N_HIP(hipGetLastError());
    M2N_HIP(hipStreamSynchronize(st));
    const double tmin = rec[0], tmax = rec[1], fmin = rec[2], fmax = rec[3];
    if (!std::isfinite(tmin) || !std::isfinite(tmax) || !std::isfinite(fmin) || !std::isfinite(fmax)) {
        set_error("non-finite sampling time or band centre");
        return M2N_ERR_ARG;
    }
    const double tc = std::rint(0.5 * (tmin + tmax));
    double X = std::max(tmax - tc, tc - tmin);
    if (!(X > 0.5)) X = 0.5;
    const double d = 1.0 / (4.0 * X);
    // kernel width of the interpolation and tolerance of the inner NuFFT: the
    // division by Psi amplifies the inner error by Psi(0) / Psi(X) (about
    // e^{0.134 beta}), so both run a decade tighter than asked
    if (tol <= 0.0) tol = prec == M2N_FP32 ? 1e-6 : 1e-12;
    int wi = (int)std::ceil(-std::log10(tol)) + 2;
    if (wi < 4) wi = 4;
    if (wi > 16) wi = 16;
    const double beta = 2.30 * wi;
    const double tol_in = prec == M2N_FP32 ? 1e-7 : std::max(tol * 0.1, 1e-14);
    const double f0 = fmin - (0.5 * wi + 2.0) * d;
    const double span_m = (fmax - fmin) / d;
    if (!(span_m < 2.0e6)) {
        set_error("band centres spread over too many grid cells for this build ((f_max - f_min) 4 X = %g)", span_m);
        return M2N_ERR_UNSUPPORTED;
    }
    const int64_t M = (int64_t)std::ceil(span_m) + wi + 5;
    if (M > (int64_t(1) << 21)) {
        set_error("type-3 grid of %lld bands exceeds 2^21", (long long)M);
        return M2N_ERR_UNSUPPORTED;
    }
    // an even Gauss-Legendre rule on [-1, 1] for Psi (as many nodes as the
    // deconvolution tables of the type-1 plans use for the same kernel and
    // the same highest frequency, w / 4); the integrand is even, so the
    // positive nodes with their weights give half the integral
    T3Quad q{};
    {
        int ng = 2 * (2 + (3 * wi + 1) / 2) + 8;
        ng += ng & 1;
        std::vector<double> gx, gw;
        gauss_legendre(ng, gx, gw);
        q.nq = 0;
        for (int j = 0; j < ng; ++j)
            if (gx[j] > 0.0) {
                q.z[q.nq] = gx[j];
                q.wq[q.nq] = gw[j];
                ++q.nq;
            }
        if (q.nq != ng / 2 || q.nq > T3_MAXQ) {
            set_error("type-3 quadrature rule of %d nodes", ng);
            return M2N_ERR_HIP;
        }
    }
    const size_t cs = prec == M2N_FP32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    const size_t b_t = ((size_t)N * 8 + 255) & ~size_t(255);
    void* wsp;
    M2N_TRY(ctx->workspace("t3_work", 2 * b_t + (size_t)K * (size_t)M * cs, &wsp));
    double* tt = (double*)wsp;
    double* xx = (double*)((char*)wsp + b_t);
    void* G = (char*)wsp + 2 * b_t;
    {
        M2N_PROF(ctx, st, "k_t3_prep");
        hipLaunchKernelGGL(k_t3_prep, dim3((unsigned)((N + T3_NT - 1) / T3_NT)), dim3(T3_NT), 0, st, t, x, N, tc,
                           (double)wi * d, beta, q, tt, xx);
    }
    M2N_HIP(hipGetLastError());
    NuSeriesIn s;
    s.t = tt;
    s.x = xx;
    s.w = w;
    s.N = N;
    s.K = K;
    s.f_lo = f0;
    s.df = d;
    s.J = G;
    M2N_TRY(nufft_run_batch(ctx, st, M, prec, tol_in, &s, 1));
    {
        M2N_PROF(ctx, st, "k_t3_interp");
        const dim3 g((unsigned)((I + T3_NT - 1) / T3_NT));
        if (prec == M2N_FP32)
            hipLaunchKernelGGL(k_t3_interp<float>, g, dim3(T3_NT), 0, st, (const cplx<float>*)G, M, K, freqs, I, f0,
                               d, wi, beta, tc, weights, (float*)P, (cplx<float>*)J);
        else
            hipLaunchKernelGGL(k_t3_interp<double>, g, dim3(T3_NT), 0, st, (const cplx<double>*)G, M, K, freqs, I,
                               f0, d, wi, beta, tc, weights, (double*)P, (cplx<double>*)J);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

}  // namespace m2n
