/*
 * m2n_oracle.c -- plain, slow, CPU FP64 reference of the M2NuFFT estimator
 * (Cui, Brinkmann & Worrell, "M2NuFFT", arXiv 2407.01943).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the GPU library, and the GPU library never calls it.
 *
 * Every routine is written straight from the paper's definitions, in FP64,
 * with no blocking, fusion or reordering beyond what the definition needs:
 *
 *   or_sinpi            sin(pi u) with exact zeros at integer u
 *   or_gpss_matrix      R(B)_{nm} = sin(2 pi f (t_n - t_m)) / (pi (t_n - t_m)),
 *                       diagonal 2 f                        (Sec. 2.1, R(B))
 *   or_band_matrix      R(A)_{nm} = sin(2 pi f_w tau)/(pi tau) e^{j 2 pi f_c tau}
 *                                                           (Sec. 2.3, R(A))
 *   or_subband_matrix   R(B^q)_{nm} = 2 cos(pi (f_max + f_min) tau)
 *                       sin(pi (f_max - f_min) tau) / (pi tau), diagonal
 *                       2 (f_max - f_min)   (Sec. 2.4, sub-band GPSS matrix)
 *   or_apply_sinc       Y = R(f) V without storing R(f)
 *   or_fft              radix-2 complex FFT (its own, for the lattice matvec)
 *   or_apply_sinc_toeplitz  Y = R(f) V for integer t as a Toeplitz
 *                       convolution on the lattice, by circular convolution
 *                       through or_fft (same numbers as or_apply_sinc up to
 *                       rounding; O(S log S) instead of O(N^2))
 *   or_cholesky         R(B) = L L^T, unblocked, row oriented
 *   or_reduce           C = L^{-1} R(A0) L^{-T}  (GEP -> standard problem)
 *   or_reduce_herm      the same for a complex Hermitian R(A0) = Ar + j Ai
 *                       and real L (sub-band GEP)
 *   or_solve_LT         X <- L^{-T} X (back substitution, several columns)
 *   or_natural_spline   natural cubic spline through (u_m, v_m), evaluated at
 *                       t_n (interpolated-DPSS tapers)
 *   or_jacobi           full eigen-decomposition by cyclic Jacobi
 *   or_lanczos          top eigenpairs of C by Lanczos with full
 *                       re-orthogonalisation (large N)
 *   or_gpss_tapers      the K largest solutions of R(A0) w = lambda R(B) w,
 *                       scaled to w^T R(B) w = 2 f_w    (Sec. 3.2 GEP at A0,
 *                       Sec. 2.2 normalisation requirement, Table 3 step 3)
 *   or_rr_select        rank-revealing reduction of a numerically singular
 *                       R(B): diagonally pivoted Cholesky, stopped when every
 *                       remaining Schur diagonal is below tau * 2 f_max; the
 *                       pivots are the samples the tapers are supported on
 *   or_nudft            J_k(A_i) = sum_n w_k(t_n) x(t_n) e^{-j 2 pi df_i t_n},
 *                       df_i = f_lo + i*df              (Sec. 3.2 eigencoeff.,
 *                       Table 3 step 4), by direct summation
 *   or_ehat_direct      D_k(i) = (E_i w_k)^* R(B) (E_i w_k),
 *                       lambda_hat = 2 f_w lambda_k / D_k(i),
 *                       Ehat_i = (1/K) sum_k |lambda_k - lambda_hat_k(i)|
 *                       (Appendix B Rayleigh quotient of shifted tapers,
 *                        Sec. 3.5 suboptimality measure)
 *
 * Parity pins for each routine live in tests/test_oracle_*.py.
 * Status codes: 0 ok, -1 bad argument, -2 t not strictly increasing,
 * -3 R(B) not positive definite, -4 no convergence.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_T_ORDER (-2)
#define OR_ERR_NOT_PD (-3)
#define OR_ERR_NO_CONVERGE (-4)

static const double OR_PI = 3.14159265358979323846264338327950288;

/* number of OpenMP threads the parallel loops use, and its setter */
int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* ------------------------------------------------------------------ */
/* argument checks (Table 3 step 1: t_n strictly increasing, 0<fw<fmax) */
/* ------------------------------------------------------------------ */
int or_validate(const double *t, long N, double fmax, double fw, int K)
{
    if (N < 1 || K < 1 || K > N) return OR_ERR_ARG;
    if (!(fmax > 0.0) || !(fw > 0.0) || !(fw < fmax)) return OR_ERR_ARG;
    if (!isfinite(fmax) || !isfinite(fw)) return OR_ERR_ARG;
    for (long n = 0; n < N; ++n)
        if (!isfinite(t[n])) return OR_ERR_ARG;
    for (long n = 1; n < N; ++n)
        if (!(t[n] > t[n - 1])) return OR_ERR_T_ORDER;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* sin(pi u): reduce u to r in [-1/2, 1/2] with sin(pi(u-2k)) = sin(pi u) */
/* and sin(pi(1-r)) = sin(pi r); every step is exact in binary64, so    */
/* integer u gives exactly 0.                                           */
/* ------------------------------------------------------------------ */
double or_sinpi(double u)
{
    double r = u - 2.0 * nearbyint(0.5 * u);   /* r in [-1, 1] */
    if (r > 0.5) r = 1.0 - r;
    else if (r < -0.5) r = -1.0 - r;
    return sin(OR_PI * r);
}

/* cos(pi u), reduced modulo 2 first (exact in binary64) */
static double or_cospi(double u)
{
    double r = u - 2.0 * nearbyint(0.5 * u);   /* r in [-1, 1] */
    return cos(OR_PI * r);
}

/* sin(2 pi f tau) / (pi tau), with the tau -> 0 limit 2 f */
static double sinc_kernel(double f, double tau)
{
    if (tau == 0.0) return 2.0 * f;
    return or_sinpi(2.0 * f * tau) / (OR_PI * tau);
}

/* R(f) as a dense N x N row-major matrix */
void or_gpss_matrix(const double *t, long N, double f, double *R)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n)
        for (long m = 0; m < N; ++m)
            R[n * N + m] = sinc_kernel(f, t[n] - t[m]);
}

/* cos/sin(2 pi u) for u given as an unevaluated sum hi + lo: reduce hi mod 1
 * exactly, then add lo. */
static void cis2pi(double hi, double lo, double *c, double *s)
{
    double r = (hi - nearbyint(hi)) + lo;
    *c = cos(2.0 * OR_PI * r);
    *s = sin(2.0 * OR_PI * r);
}

/* complex band matrix R(A)_{nm} for the band centred at fc, half-width fw */
void or_band_matrix(const double *t, long N, double fc, double fw,
                    double *Rre, double *Rim)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n)
        for (long m = 0; m < N; ++m) {
            double tau = t[n] - t[m];
            double a = sinc_kernel(fw, tau);
            double hi = fc * tau, lo = fma(fc, tau, -hi), c, s;
            cis2pi(hi, lo, &c, &s);
            Rre[n * N + m] = a * c;
            Rim[n * N + m] = a * s;
        }
}

/* R(B^q) of the sub-band f_min <= |f| <= f_max as a dense N x N row-major
 * matrix: the integral of e^{j 2 pi f tau} over both halves of the sub-band,
 * 2 cos(pi (f_max + f_min) tau) sin(pi (f_max - f_min) tau) / (pi tau). */
void or_subband_matrix(const double *t, long N, double fmin, double fmax, double *R)
{
    const double fs = fmax + fmin, fd = fmax - fmin;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n)
        for (long m = 0; m < N; ++m) {
            double tau = t[n] - t[m];
            R[n * N + m] = (tau == 0.0) ? 2.0 * fd
                : 2.0 * or_cospi(fs * tau) * or_sinpi(fd * tau) / (OR_PI * tau);
        }
}

/* Y (N x nv, row-major) = R(f) V (N x nv, row-major), R generated on the fly.
 * When every t_n is an integer the kernel values are looked up in a table of
 * integer lags (the same numbers, computed once). */
void or_apply_sinc(const double *t, long N, double f, const double *V,
                   long nv, double *Y)
{
    int integral = 1;
    for (long n = 0; n < N; ++n)
        if (t[n] != nearbyint(t[n]) || fabs(t[n]) > 1e15) { integral = 0; break; }
    double *lag = NULL;
    long span = 0;
    if (integral && N > 0) {
        span = (long)(t[N - 1] - t[0]);
        lag = (double *)malloc(sizeof(double) * (size_t)(span + 1));
        for (long j = 0; j <= span; ++j) lag[j] = sinc_kernel(f, (double)j);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (long n = 0; n < N; ++n) {
        double *y = Y + n * nv;
        for (long c = 0; c < nv; ++c) y[c] = 0.0;
        for (long m = 0; m < N; ++m) {
            double r;
            if (lag) {
                long j = (long)(t[n] - t[m]);
                r = lag[j < 0 ? -j : j];
            } else {
                r = sinc_kernel(f, t[n] - t[m]);
            }
            const double *v = V + m * nv;
            for (long c = 0; c < nv; ++c) y[c] += r * v[c];
        }
    }
    free(lag);
}

/* ------------------------------------------------------------------ */
/* Radix-2 complex FFT in place, M a power of two:                      */
/*   X_k = sum_j x_j exp(sgn * 2 pi i j k / M)                          */
/* Iterative Cooley-Tukey: bit-reversal permutation, then log2(M)       */
/* butterfly stages; each twiddle is the cosine and sine of the exact    */
/* fraction k / len (reduced as in or_sinpi).                            */
/* ------------------------------------------------------------------ */
void or_fft(double *re, double *im, long M, int sgn)
{
    for (long i = 1, j = 0; i < M; ++i) {
        long bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double a = re[i]; re[i] = re[j]; re[j] = a;
            a = im[i]; im[i] = im[j]; im[j] = a;
        }
    }
    for (long len = 2; len <= M; len <<= 1) {
        long half = len / 2;
        for (long k = 0; k < half; ++k) {
            double u = 2.0 * (double)k / (double)len;
            double c = or_cospi(u), sn = (sgn < 0 ? -1.0 : 1.0) * or_sinpi(u);
            for (long b = 0; b < M; b += len) {
                long p0 = b + k, q0 = p0 + half;
                double tr = re[q0] * c - im[q0] * sn;
                double ti = re[q0] * sn + im[q0] * c;
                re[q0] = re[p0] - tr;
                im[q0] = im[p0] - ti;
                re[p0] += tr;
                im[p0] += ti;
            }
        }
    }
}

/* R(f) on an integer lattice as a Toeplitz operator: with o_n = t_n - t_0
 * and S = o_{N-1}, (R v)_n = sum_m h(o_n - o_m) v_m, h(j) = sin(2 pi f j)/(pi j),
 * i.e. the linear convolution of h (lags -S..S) with v placed on the lattice
 * (zeros at the missing points), sampled at the o_n.  A circular
 * convolution of length M >= 2 S + 1 holds it exactly; H = FFT(h) is
 * computed once per operator. */
typedef struct {
    long N, S, M;
    long *o;
    double *Hr, *Hi, *wr, *wi;
} toep_op;

static int toep_init(toep_op *op, const double *t, long N, double f)
{
    memset(op, 0, sizeof(*op));
    for (long n = 0; n < N; ++n)
        if (t[n] != nearbyint(t[n]) || fabs(t[n]) > 1e15) return OR_ERR_ARG;
    for (long n = 1; n < N; ++n)
        if (!(t[n] > t[n - 1])) return OR_ERR_T_ORDER;
    long S = (long)(t[N - 1] - t[0]);
    long M = 1;
    while (M < 2 * S + 1) M <<= 1;
    op->N = N;
    op->S = S;
    op->M = M;
    op->o = (long *)malloc(sizeof(long) * (size_t)N);
    op->Hr = (double *)calloc((size_t)M, sizeof(double));
    op->Hi = (double *)calloc((size_t)M, sizeof(double));
    op->wr = (double *)malloc(sizeof(double) * (size_t)M);
    op->wi = (double *)malloc(sizeof(double) * (size_t)M);
    for (long n = 0; n < N; ++n) op->o[n] = (long)(t[n] - t[0]);
    op->Hr[0] = sinc_kernel(f, 0.0);
    for (long j = 1; j <= S; ++j) {
        double h = sinc_kernel(f, (double)j);
        op->Hr[j] = h;
        op->Hr[M - j] = h;
    }
    or_fft(op->Hr, op->Hi, M, -1);
    return OR_OK;
}

static void toep_apply(const toep_op *op, const double *v, long stride, double *y, long ystride)
{
    const long M = op->M;
    memset(op->wr, 0, sizeof(double) * (size_t)M);
    memset(op->wi, 0, sizeof(double) * (size_t)M);
    for (long n = 0; n < op->N; ++n) op->wr[op->o[n]] = v[n * stride];
    or_fft(op->wr, op->wi, M, -1);
    for (long k = 0; k < M; ++k) {
        double a = op->wr[k], b = op->wi[k];
        op->wr[k] = a * op->Hr[k] - b * op->Hi[k];
        op->wi[k] = a * op->Hi[k] + b * op->Hr[k];
    }
    or_fft(op->wr, op->wi, M, +1);
    for (long n = 0; n < op->N; ++n) y[n * ystride] = op->wr[op->o[n]] / (double)M;
}

static void toep_free(toep_op *op)
{
    free(op->o); free(op->Hr); free(op->Hi); free(op->wr); free(op->wi);
    memset(op, 0, sizeof(*op));
}

/* Y (N x nv, row-major) = R(f) V for strictly increasing integer t, through
 * the lattice Toeplitz operator.  Returns 0, or OR_ERR_ARG for non-integer t. */
int or_apply_sinc_toeplitz(const double *t, long N, double f, const double *V,
                           long nv, double *Y)
{
    toep_op op;
    int st = toep_init(&op, t, N, f);
    if (st) { toep_free(&op); return st; }
    for (long c = 0; c < nv; ++c) toep_apply(&op, V + c, nv, Y + c, nv);
    toep_free(&op);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Cholesky R = L L^T (lower, row-major, in place; upper part zeroed)  */
/* returns 0 or -(index of the failing pivot + 1)                      */
/* ------------------------------------------------------------------ */
long or_cholesky(double *A, long N)
{
    for (long j = 0; j < N; ++j) {
        double d = A[j * N + j];
        for (long k = 0; k < j; ++k) d -= A[j * N + k] * A[j * N + k];
        if (!(d > 0.0)) return -(j + 1);
        double ljj = sqrt(d);
        A[j * N + j] = ljj;
#pragma omp parallel for schedule(static)
        for (long i = j + 1; i < N; ++i) {
            double s = A[i * N + j];
            for (long k = 0; k < j; ++k) s -= A[i * N + k] * A[j * N + k];
            A[i * N + j] = s / ljj;
        }
    }
    for (long i = 0; i < N; ++i)
        for (long j = i + 1; j < N; ++j) A[i * N + j] = 0.0;
    return 0;
}

/* solve L z = b in place (forward substitution), row-major L */
static void fwd_subst(const double *L, long N, double *b, long stride)
{
    for (long i = 0; i < N; ++i) {
        double s = b[i * stride];
        for (long k = 0; k < i; ++k) s -= L[i * N + k] * b[k * stride];
        b[i * stride] = s / L[i * N + i];
    }
}

/* solve L^T z = b in place (back substitution) */
static void back_subst_T(const double *L, long N, double *b, long stride)
{
    for (long i = N - 1; i >= 0; --i) {
        double s = b[i * stride];
        for (long k = i + 1; k < N; ++k) s -= L[k * N + i] * b[k * stride];
        b[i * stride] = s / L[i * N + i];
    }
}

/* C = L^{-1} RA L^{-T}, symmetrised; all N x N row-major */
void or_reduce(const double *L, const double *RA, long N, double *C)
{
    double *M = (double *)malloc(sizeof(double) * (size_t)N * (size_t)N);
    memcpy(M, RA, sizeof(double) * (size_t)N * (size_t)N);
    /* M <- L^{-1} RA : forward-substitute every column */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) fwd_subst(L, N, M + c, N);
    /* C <- M L^{-T} = (L^{-1} M^T)^T : forward-substitute every row of M */
#pragma omp parallel for schedule(static)
    for (long r = 0; r < N; ++r) fwd_subst(L, N, M + r * N, 1);
    for (long i = 0; i < N; ++i)
        for (long j = 0; j < N; ++j)
            C[i * N + j] = 0.5 * (M[i * N + j] + M[j * N + i]);
    free(M);
}

/* Complex Hermitian R(A0) = Ar + j Ai (Ar symmetric, Ai antisymmetric)
 * with real L: C = L^{-1} R(A0) L^{-T} has real part L^{-1} Ar L^{-T}
 * (symmetrised) and imaginary part L^{-1} Ai L^{-T} (antisymmetrised). */
void or_reduce_herm(const double *L, const double *Ar, const double *Ai, long N,
                    double *Cr, double *Ci)
{
    size_t NN = (size_t)N * (size_t)N;
    double *M = (double *)malloc(sizeof(double) * NN);
    for (int part = 0; part < 2; ++part) {
        memcpy(M, part ? Ai : Ar, sizeof(double) * NN);
#pragma omp parallel for schedule(static)
        for (long c = 0; c < N; ++c) fwd_subst(L, N, M + c, N);
#pragma omp parallel for schedule(static)
        for (long r = 0; r < N; ++r) fwd_subst(L, N, M + r * N, 1);
        double *C = part ? Ci : Cr;
        double sg = part ? -1.0 : 1.0;
        for (long i = 0; i < N; ++i)
            for (long j = 0; j < N; ++j)
                C[i * N + j] = 0.5 * (M[i * N + j] + sg * M[j * N + i]);
    }
    free(M);
}

/* X (N x nrhs, row-major) <- L^{-T} X */
void or_solve_LT(const double *L, long N, double *X, long nrhs)
{
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nrhs; ++c) back_subst_T(L, N, X + c, nrhs);
}

/* Natural cubic spline through (u_m, v_m), m < n (u strictly increasing,
 * n >= 2), evaluated at x[0..nx): second derivatives M with M_0 = M_{n-1} = 0
 * from the continuity of the first derivative at the interior knots,
 *   h_{m-1} M_{m-1} + 2 (h_{m-1} + h_m) M_m + h_m M_{m+1}
 *       = 6 ((v_{m+1} - v_m) / h_m - (v_m - v_{m-1}) / h_{m-1}),
 * solved by forward elimination and back substitution (the system is
 * tridiagonal and diagonally dominant); on [u_m, u_{m+1}] the cubic is
 *   M_m (u_{m+1} - x)^3 / (6 h) + M_{m+1} (x - u_m)^3 / (6 h)
 *   + (v_m / h - M_m h / 6) (u_{m+1} - x) + (v_{m+1} / h - M_{m+1} h / 6) (x - u_m).
 * Points outside [u_0, u_{n-1}] use the end intervals' cubics.  nv series
 * v[k * n + m] share the knots; out[k * nx + i]. */
void or_natural_spline(const double *u, long n, const double *v, long nv,
                       const double *x, long nx, double *out)
{
    double *M = (double *)calloc((size_t)n, sizeof(double));
    double *cp = (double *)calloc((size_t)n, sizeof(double));
    double *dp = (double *)calloc((size_t)n, sizeof(double));
    for (long k = 0; k < nv; ++k) {
        const double *vk = v + k * n;
        for (long m = 0; m < n; ++m) M[m] = 0.0;
        if (n > 2) {
            /* unknowns M_1..M_{n-2}; row m: a M_{m-1} + b M_m + c M_{m+1} = d */
            for (long m = 1; m <= n - 2; ++m) {
                double h0 = u[m] - u[m - 1], h1 = u[m + 1] - u[m];
                double a = h0, b = 2.0 * (h0 + h1), c = h1;
                double d = 6.0 * ((vk[m + 1] - vk[m]) / h1 - (vk[m] - vk[m - 1]) / h0);
                if (m > 1) {
                    double den = b - a * cp[m - 1];
                    cp[m] = c / den;
                    dp[m] = (d - a * dp[m - 1]) / den;
                } else {
                    cp[m] = c / b;
                    dp[m] = d / b;
                }
            }
            M[n - 2] = dp[n - 2];
            for (long m = n - 3; m >= 1; --m) M[m] = dp[m] - cp[m] * M[m + 1];
        }
        for (long i = 0; i < nx; ++i) {
            double xi = x[i];
            long lo = 0, hi = n - 1;            /* u[lo] <= xi < u[hi] */
            while (hi - lo > 1) {
                long mid = (lo + hi) / 2;
                if (u[mid] <= xi) lo = mid; else hi = mid;
            }
            double h = u[hi] - u[lo], A = u[hi] - xi, B = xi - u[lo];
            out[k * nx + i] = M[lo] * A * A * A / (6.0 * h) + M[hi] * B * B * B / (6.0 * h)
                              + (vk[lo] / h - M[lo] * h / 6.0) * A
                              + (vk[hi] / h - M[hi] * h / 6.0) * B;
        }
    }
    free(M); free(cp); free(dp);
}

/* ------------------------------------------------------------------ */
/* Cyclic Jacobi with a threshold, for a symmetric N x N row-major A.  */
/* On return evals[] is sorted in descending order and column k of V   */
/* (V[n*N+k]) is the unit eigenvector for evals[k].  A is destroyed.   */
/* Returns the number of sweeps, or OR_ERR_NO_CONVERGE.                */
/* ------------------------------------------------------------------ */
int or_jacobi(double *A, long N, double *evals, double *V, int max_sweeps)
{
    for (long i = 0; i < N; ++i)
        for (long j = 0; j < N; ++j) V[i * N + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (long i = 0; i < N * N; ++i) fro += A[i] * A[i];
    fro = sqrt(fro);
    int sweep;
    int converged = (N <= 1);
    for (sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        double off = 0.0;
        for (long i = 0; i < N; ++i)
            for (long j = i + 1; j < N; ++j) off += A[i * N + j] * A[i * N + j];
        off = sqrt(2.0 * off);
        if (off <= 1e-15 * fro || off == 0.0) { converged = 1; break; }
        double thresh = (sweep < 3) ? 0.2 * off / (double)(N * N) : 0.0;
        for (long p = 0; p < N - 1; ++p) {
            for (long q = p + 1; q < N; ++q) {
                double apq = A[p * N + q];
                if (fabs(apq) <= thresh || apq == 0.0) continue;
                double app = A[p * N + p], aqq = A[q * N + q];
                double theta = (aqq - app) / (2.0 * apq);
                double tt = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) tt = -tt;
                double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
                double tau = s / (1.0 + c);
                A[p * N + p] = app - tt * apq;
                A[q * N + q] = aqq + tt * apq;
                A[p * N + q] = A[q * N + p] = 0.0;
                for (long r = 0; r < N; ++r) {
                    if (r == p || r == q) continue;
                    double arp = A[r * N + p], arq = A[r * N + q];
                    double nrp = arp - s * (arq + tau * arp);
                    double nrq = arq + s * (arp - tau * arq);
                    A[r * N + p] = A[p * N + r] = nrp;
                    A[r * N + q] = A[q * N + r] = nrq;
                }
                for (long r = 0; r < N; ++r) {
                    double vrp = V[r * N + p], vrq = V[r * N + q];
                    V[r * N + p] = vrp - s * (vrq + tau * vrp);
                    V[r * N + q] = vrq + s * (vrp - tau * vrq);
                }
            }
        }
    }
    if (!converged) {
        double off = 0.0;
        for (long i = 0; i < N; ++i)
            for (long j = i + 1; j < N; ++j) off += A[i * N + j] * A[i * N + j];
        if (sqrt(2.0 * off) > 1e-15 * fro && off != 0.0) return OR_ERR_NO_CONVERGE;
    }
    /* selection sort, descending, columns of V follow */
    for (long i = 0; i < N; ++i) evals[i] = A[i * N + i];
    for (long i = 0; i < N; ++i) {
        long best = i;
        for (long j = i + 1; j < N; ++j)
            if (evals[j] > evals[best]) best = j;
        if (best != i) {
            double tmp = evals[i]; evals[i] = evals[best]; evals[best] = tmp;
            for (long r = 0; r < N; ++r) {
                double v = V[r * N + i]; V[r * N + i] = V[r * N + best]; V[r * N + best] = v;
            }
        }
    }
    return sweep;
}

/* ------------------------------------------------------------------ */
/* Sign convention (the paper leaves it open): with s1 = sum_n w_n and */
/* s2 = sum_n (tbar - t_n) w_n / (t_N - t_1), tbar = (t_1 + t_N)/2, the */
/* one of larger magnitude is made positive ("even tapers sum positive, */
/* odd tapers start positive").                                         */
/* ------------------------------------------------------------------ */
static void fix_sign(const double *t, long N, double *w)
{
    double s1 = 0.0, s2 = 0.0;
    double span = (N > 1) ? (t[N - 1] - t[0]) : 1.0;
    double tbar = 0.5 * (t[0] + t[N - 1]);
    for (long n = 0; n < N; ++n) {
        s1 += w[n];
        s2 += (tbar - t[n]) * w[n] / span;
    }
    double key = (fabs(s1) >= fabs(s2)) ? s1 : s2;
    if (key < 0.0)
        for (long n = 0; n < N; ++n) w[n] = -w[n];
}

/* ------------------------------------------------------------------ */
/* Lanczos with full re-orthogonalisation for the largest eigenpairs of */
/* C = L^{-1} R(A0) L^{-T}.  L == NULL means L = sqrt(cdiag) I.         */
/* toeplitz != 0 (with L == NULL and integer t): R(A0) is applied as the */
/* lattice Toeplitz convolution instead of the direct O(N^2) sum.       */
/* Ritz pairs come from the Jacobi decomposition of the tridiagonal T.  */
/* y is N x nwant row-major (column k = unit Ritz vector k).            */
/* ------------------------------------------------------------------ */
static void apply_C(const double *t, long N, double fw, const double *L,
                    double cdiag, const toep_op *op, const double *v, double *out,
                    double *tmp)
{
    memcpy(tmp, v, sizeof(double) * (size_t)N);
    if (L) back_subst_T(L, N, tmp, 1);
    else for (long n = 0; n < N; ++n) tmp[n] /= sqrt(cdiag);
    if (op) toep_apply(op, tmp, 1, out, 1);
    else or_apply_sinc(t, N, fw, tmp, 1, out);
    if (L) fwd_subst(L, N, out, 1);
    else for (long n = 0; n < N; ++n) out[n] /= sqrt(cdiag);
}

int or_lanczos(const double *t, long N, double fw, const double *L,
               double cdiag, int nwant, int mmax, double tol,
               double *evals, double *y, uint64_t seed, int toeplitz)
{
    if (mmax > N) mmax = (int)N;
    if (nwant > mmax) return OR_ERR_ARG;
    toep_op op_store, *op = NULL;
    if (toeplitz) {
        if (L) return OR_ERR_ARG;
        int st0 = toep_init(&op_store, t, N, fw);
        if (st0) { toep_free(&op_store); return st0; }
        op = &op_store;
    }
    double *Q = (double *)calloc((size_t)(mmax + 1) * (size_t)N, sizeof(double));
    double *z = (double *)malloc(sizeof(double) * (size_t)N);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)N);
    double *alpha = (double *)calloc((size_t)mmax + 1, sizeof(double));
    double *beta = (double *)calloc((size_t)mmax + 1, sizeof(double));
    double *T = (double *)malloc(sizeof(double) * (size_t)mmax * (size_t)mmax);
    double *S = (double *)malloc(sizeof(double) * (size_t)mmax * (size_t)mmax);
    double *th = (double *)malloc(sizeof(double) * (size_t)mmax);
    int status = OR_ERR_NO_CONVERGE, m_used = 0;
    /* deterministic start vector: splitmix64 -> uniform(-1,1) */
    uint64_t st = seed;
    double nrm = 0.0;
    for (long n = 0; n < N; ++n) {
        uint64_t zz = (st += 0x9E3779B97F4A7C15ull);
        zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
        zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
        zz ^= zz >> 31;
        Q[n] = ((double)(zz >> 11) / 9007199254740992.0) * 2.0 - 1.0;
        nrm += Q[n] * Q[n];
    }
    nrm = sqrt(nrm);
    for (long n = 0; n < N; ++n) Q[n] /= nrm;
    for (int j = 0; j < mmax; ++j) {
        double *qj = Q + (size_t)j * N;
        apply_C(t, N, fw, L, cdiag, op, qj, z, tmp);
        double a = 0.0;
        for (long n = 0; n < N; ++n) a += qj[n] * z[n];
        alpha[j] = a;
        /* full re-orthogonalisation, twice */
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i <= j; ++i) {
                double *qi = Q + (size_t)i * N, d = 0.0;
                for (long n = 0; n < N; ++n) d += qi[n] * z[n];
                for (long n = 0; n < N; ++n) z[n] -= d * qi[n];
            }
        double b = 0.0;
        for (long n = 0; n < N; ++n) b += z[n] * z[n];
        b = sqrt(b);
        beta[j] = b;
        m_used = j + 1;
        int check = (m_used >= nwant) && ((m_used % 8 == 0) || m_used == mmax || b < 1e-300);
        if (check) {
            int m = m_used;
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) {
                    double v = 0.0;
                    if (r == c) v = alpha[r];
                    else if (c == r + 1) v = beta[r];
                    else if (r == c + 1) v = beta[c];
                    T[r * m + c] = v;
                }
            if (or_jacobi(T, m, th, S, 100) < 0) break;
            double worst = 0.0;
            for (int k = 0; k < nwant; ++k) {
                double res = fabs(b * S[(m - 1) * m + k]);
                if (res > worst) worst = res;
            }
            if (worst <= tol || b < 1e-300 || m == mmax) {
                for (int k = 0; k < nwant; ++k) evals[k] = th[k];
                for (long n = 0; n < N; ++n)
                    for (int k = 0; k < nwant; ++k) {
                        double s = 0.0;
                        for (int i = 0; i < m; ++i) s += Q[(size_t)i * N + n] * S[i * m + k];
                        y[n * nwant + k] = s;
                    }
                status = (worst <= tol || b < 1e-300) ? m : OR_ERR_NO_CONVERGE;
                break;
            }
        }
        if (b < 1e-300) break;
        double *qn = Q + (size_t)(j + 1) * N;
        for (long n = 0; n < N; ++n) qn[n] = z[n] / b;
    }
    free(Q); free(z); free(tmp); free(alpha); free(beta); free(T); free(S); free(th);
    if (op) toep_free(op);
    return status;
}

/* ------------------------------------------------------------------ */
/* The K largest GPSS tapers at the nominal band A0 (f_c0 = 0):        */
/*   R(A0) w = lambda R(B) w,  w_k^T R(B) w_k = 2 f_w.                 */
/* method 0: dense reduction + Jacobi; 1: Lanczos; 2: Lanczos on an   */
/* integer lattice with integer 2 f_max (R(B) = 2 f_max I, Toeplitz     */
/* R(A0), no N x N matrix).                                            */
/* w is K x N row-major, lam[K] descending.                            */
/* ------------------------------------------------------------------ */
long or_gpss_tapers(const double *t, long N, double fmax, double fw, int K,
                    int method, double *w, double *lam)
{
    int st = or_validate(t, N, fmax, fw, K);
    if (st) return st;
    if (method == 2) {
        /* integer lattice with integer 2 f_max: every off-diagonal
         * sin(2 pi f_max tau) of R(B) is an exact zero, R(B) = 2 f_max I; the
         * GEP is the standard problem of R(A0) / (2 f_max), solved by Lanczos
         * with the Toeplitz operator (no N x N matrix is formed) */
        double cB = 2.0 * fmax;
        if (cB != nearbyint(cB) || cB < 1.0) return OR_ERR_ARG;
        for (long n = 0; n < N; ++n)
            if (t[n] != nearbyint(t[n]) || fabs(t[n]) > 1e15) return OR_ERR_ARG;
        double *y = (double *)malloc(sizeof(double) * (size_t)N * (size_t)K);
        int mmax = (int)((N < 400) ? N : 400);
        int sw = or_lanczos(t, N, fw, NULL, cB, K, mmax, 1e-14, lam, y, 0x5EEDull, 1);
        double *col = (double *)malloc(sizeof(double) * (size_t)N);
        for (int k = 0; k < K; ++k) {
            for (long n = 0; n < N; ++n) col[n] = y[n * K + k] / sqrt(cB) * sqrt(2.0 * fw);
            fix_sign(t, N, col);
            memcpy(w + (size_t)k * N, col, sizeof(double) * (size_t)N);
        }
        free(col); free(y);
        return sw < 0 ? OR_ERR_NO_CONVERGE : 0;
    }
    size_t NN = (size_t)N * (size_t)N;
    double *RB = (double *)malloc(sizeof(double) * NN);
    or_gpss_matrix(t, N, fmax, RB);
    /* a diagonal R(B) (e.g. the integer lattice with f_max = 1/2) has the
     * trivial factor sqrt(diag); it is detected, not assumed */
    int diagonal = 1;
    for (long n = 0; n < N && diagonal; ++n)
        for (long m = 0; m < N; ++m)
            if (n != m && RB[n * N + m] != 0.0) { diagonal = 0; break; }
    long chol = 0;
    if (!diagonal) chol = or_cholesky(RB, N);
    if (chol < 0) { free(RB); return OR_ERR_NOT_PD; }
    double cdiag = 2.0 * fmax;
    double *y = (double *)malloc(sizeof(double) * (size_t)N * (size_t)K);
    long ret = 0;
    if (method == 0) {
        double *RA = (double *)malloc(sizeof(double) * NN);
        double *C = (double *)malloc(sizeof(double) * NN);
        double *V = (double *)malloc(sizeof(double) * NN);
        double *ev = (double *)malloc(sizeof(double) * (size_t)N);
        or_gpss_matrix(t, N, fw, RA);
        if (diagonal) {
            for (size_t i = 0; i < NN; ++i) C[i] = RA[i] / cdiag;
        } else {
            or_reduce(RB, RA, N, C);
        }
        int sw = or_jacobi(C, N, ev, V, 100);
        if (sw < 0) ret = OR_ERR_NO_CONVERGE;
        for (int k = 0; k < K; ++k) {
            lam[k] = ev[k];
            for (long n = 0; n < N; ++n) y[n * K + k] = V[n * N + k];
        }
        free(RA); free(C); free(V); free(ev);
    } else {
        int mmax = (int)((N < 400) ? N : 400);
        int sw = or_lanczos(t, N, fw, diagonal ? NULL : RB, cdiag, K, mmax,
                            1e-14, lam, y, 0x5EEDull, 0);
        if (sw < 0) ret = OR_ERR_NO_CONVERGE;
    }
    /* w_k = sqrt(2 f_w) L^{-T} y_k  =>  w_k^T R(B) w_k = 2 f_w */
    double *col = (double *)malloc(sizeof(double) * (size_t)N);
    for (int k = 0; k < K; ++k) {
        for (long n = 0; n < N; ++n) col[n] = y[n * K + k];
        if (diagonal) for (long n = 0; n < N; ++n) col[n] /= sqrt(cdiag);
        else back_subst_T(RB, N, col, 1);
        for (long n = 0; n < N; ++n) col[n] *= sqrt(2.0 * fw);
        fix_sign(t, N, col);
        memcpy(w + (size_t)k * N, col, sizeof(double) * (size_t)N);
    }
    free(col); free(y); free(RB);
    return ret;
}

/* ------------------------------------------------------------------ */
/* Rank-revealing reduction (no positive-definiteness assumed):         */
/* R(B) = P L L^T P^T + S with diagonal pivoting; at each step the       */
/* sample with the largest remaining Schur diagonal d_i is taken (ties,   */
/* i.e. d_i >= (1 - 1e-12) max d, go to the smallest index), and the      */
/* process stops when max d < tau * 2 f_max.  sel[n] = 1 for the taken     */
/* samples; returns their number r; *maxrem = the largest remaining d.   */
/* The columns of L are formed from their definition,                     */
/*   l_{i,j} = (R_{i,p} - sum_{k<j} l_{i,k} l_{p,k}) / sqrt(d_p).          */
/* ------------------------------------------------------------------ */
long or_rr_select(const double *t, long N, double fmax, double tau, int *sel, double *maxrem)
{
    double *d = (double *)malloc(sizeof(double) * (size_t)N);
    double *L = (double *)calloc((size_t)N * (size_t)N, sizeof(double));   /* column j at L + j N */
    long *piv = (long *)malloc(sizeof(long) * (size_t)N);
    const double dmax0 = 2.0 * fmax;
    for (long i = 0; i < N; ++i) { d[i] = dmax0; sel[i] = 0; }
    long r = 0;
    for (long j = 0; j < N; ++j) {
        double mx = -1.0;
        for (long i = 0; i < N; ++i)
            if (!sel[i] && d[i] > mx) mx = d[i];
        if (!(mx >= tau * dmax0)) break;
        long p = -1;
        for (long i = 0; i < N && p < 0; ++i)
            if (!sel[i] && d[i] >= (1.0 - 1e-12) * mx) p = i;
        sel[p] = 1;
        piv[j] = p;
        const double sp = sqrt(d[p]);
        double *lj = L + (size_t)j * (size_t)N;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            if (sel[i] && i != p) { lj[i] = 0.0; continue; }
            double v = sinc_kernel(fmax, t[i] - t[p]);
            for (long k = 0; k < j; ++k) v -= L[(size_t)k * N + i] * L[(size_t)k * N + p];
            lj[i] = v / sp;
        }
        for (long i = 0; i < N; ++i)
            if (!sel[i]) d[i] -= lj[i] * lj[i];
        d[p] = 0.0;
        r = j + 1;
    }
    double mr = 0.0;
    for (long i = 0; i < N; ++i)
        if (!sel[i] && d[i] > mr) mr = d[i];
    *maxrem = mr;
    free(d); free(L); free(piv);
    return r;
}

/* ------------------------------------------------------------------ */
/* Direct NUDFT (eigencoefficients), compensated phase:                */
/*   J_k(i) = sum_n w_k(t_n) x_n exp(-j 2 pi (f_lo + i df) t_n)         */
/* for the band indices bands[0..nb).  J is K x nb (re, im separate).  */
/* The phase (f_lo + i df) t_n is formed from exact two-products and   */
/* reduced modulo 1 before the cosine/sine.                            */
/* ------------------------------------------------------------------ */
static void band_phasor(double f_lo, double df, long i, double tn,
                        double *c, double *s)
{
    double a_hi = f_lo * tn, a_lo = fma(f_lo, tn, -a_hi);
    double d_hi = df * tn, d_lo = fma(df, tn, -d_hi);
    double di = (double)i;
    double b_hi = di * d_hi, b_lo = fma(di, d_hi, -b_hi) + di * d_lo;
    double hi = (a_hi - nearbyint(a_hi)) + (b_hi - nearbyint(b_hi));
    double lo = a_lo + b_lo;
    cis2pi(hi, lo, c, s);
}

void or_nudft(const double *t, const double *x, const double *w, long N,
              int K, double f_lo, double df, const long *bands, long nb,
              double *Jre, double *Jim)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long b = 0; b < nb; ++b) {
        long i = bands[b];
        double acc_re[64], acc_im[64];
        for (int k = 0; k < K; ++k) { acc_re[k] = 0.0; acc_im[k] = 0.0; }
        for (long n = 0; n < N; ++n) {
            double c, s;
            band_phasor(f_lo, df, i, t[n], &c, &s);
            /* e^{-j 2 pi phase} = c - j s */
            for (int k = 0; k < K; ++k) {
                double a = w[(size_t)k * N + n] * x[n];
                acc_re[k] += a * c;
                acc_im[k] -= a * s;
            }
        }
        for (int k = 0; k < K; ++k) {
            Jre[(size_t)k * nb + b] = acc_re[k];
            Jim[(size_t)k * nb + b] = acc_im[k];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Suboptimality estimate by the direct quadratic form.                */
/*   z = E_i w_k,  E_i = diag(exp(+j 2 pi df_i t_n))                    */
/*   D_k(i) = z^* R(B) z,  lambda_hat = 2 f_w lambda_k / D_k(i)          */
/*   Ehat_i = (1/K) sum_k |lambda_k - lambda_hat_k(i)|                  */
/* D is K x nb, E is nb.                                               */
/* ------------------------------------------------------------------ */
void or_ehat_direct(const double *t, const double *w, const double *lam,
                    long N, int K, double fmax, double fw, double f_lo,
                    double df, const long *bands, long nb, double *D,
                    double *E)
{
    size_t NN = (size_t)N * (size_t)N;
    double *RB = (double *)malloc(sizeof(double) * NN);
    or_gpss_matrix(t, N, fmax, RB);
#pragma omp parallel for schedule(dynamic, 1)
    for (long b = 0; b < nb; ++b) {
        long i = bands[b];
        double *zr = (double *)malloc(sizeof(double) * (size_t)N);
        double *zi = (double *)malloc(sizeof(double) * (size_t)N);
        double esum = 0.0;
        for (int k = 0; k < K; ++k) {
            for (long n = 0; n < N; ++n) {
                double c, s;
                band_phasor(f_lo, df, i, t[n], &c, &s);
                zr[n] = w[(size_t)k * N + n] * c;   /* w e^{+j...} */
                zi[n] = w[(size_t)k * N + n] * s;
            }
            double acc = 0.0;
            for (long n = 0; n < N; ++n) {
                double yr = 0.0, yi = 0.0;
                const double *row = RB + (size_t)n * N;
                for (long m = 0; m < N; ++m) {
                    yr += row[m] * zr[m];
                    yi += row[m] * zi[m];
                }
                acc += zr[n] * yr + zi[n] * yi;   /* Re(conj(z_n) y_n) */
            }
            D[(size_t)k * nb + b] = acc;
            double lh = 2.0 * fw * lam[k] / acc;
            esum += fabs(lam[k] - lh);
        }
        E[b] = esum / (double)K;
        free(zr); free(zi);
    }
    free(RB);
}
