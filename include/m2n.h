/*
 * m2n.h -- C-ABI of the MI355X M2NuFFT library (libm2n.so).
 *
 * The estimator (Cui, Brinkmann & Worrell, M2NuFFT, arXiv 2407.01943) for a
 * gapped or nonuniformly sampled series x(t_n), n = 1..N, with signal band
 * B = [-f_max, f_max], nominal analysis band A0 = [-f_w, f_w] and I analysis
 * bands A_i centred at f_lo + i*df:
 *
 *   tapers     R(A0) w_k = lambda_k R(B) w_k, the K largest, scaled so that
 *              w_k^T R(B) w_k = 2 f_w              (Sec. 3.2 GEP at A0, Sec. 2.2
 *                                                   normalisation; Table 3 step 3)
 *   eigcoeffs  J_k(A_i) = sum_n w_k(t_n) x(t_n) exp(-j 2 pi (f_lo + i df) t_n)
 *                                                  (Sec. 3.2; Table 3 step 4)
 *   psd        P(A_i) = sum_k d_k |J_k(A_i)|^2, d_k = 1/K by default
 *                                                  (Sec. 3.2; Table 3 step 5)
 *   ehat       Ehat_i = (1/K) sum_k |lambda_k - 2 f_w lambda_k / D_k(i)|,
 *              D_k(i) = (E_i w_k)^* R(B) (E_i w_k)  (Sec. 3.5 with the
 *                                                   Appendix B Rayleigh quotient)
 *
 * R(B)_{nm} = sin(2 pi f_max tau)/(pi tau), R(A0)_{nm} = sin(2 pi f_w tau)/(pi tau),
 * tau = t_n - t_m (Sec. 2.1, Sec. 2.3); the diagonals are 2 f_max and 2 f_w.
 *
 * Conventions for every call below
 *  - Every array argument is a DEVICE pointer (HIP device memory of the
 *    context's device) owned by the caller; the library never frees it and
 *    keeps no reference after the call's stream work has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Layouts are row-major: tapers w are K x N (taper k at w + k*N), the
 *    eigencoefficients J are K x I complex (interleaved re, im).
 *  - Sizes are int64_t; N >= 1, 1 <= K <= min(N, 64), 1 <= I <= 2^21.
 *  - Errors are returned as m2n_status codes; nothing aborts and no C++
 *    exception crosses the ABI.  m2n_last_error(ctx) gives a text for the last
 *    failure on the calling thread.
 *  - A context is not thread-safe: one host thread at a time per context.
 *    Its workspace is reused from call to call, so calls on one context
 *    must be ordered: one stream, or the caller synchronises between them.
 */
#ifndef M2N_H
#define M2N_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct m2n_ctx m2n_ctx;

typedef enum {
    M2N_OK = 0,
    M2N_ERR_ARG = -1,          /* bad size, NULL pointer or non-finite value     */
    M2N_ERR_T_ORDER = -2,      /* sampling times not strictly increasing         */
    M2N_ERR_NOT_PD = -3,       /* R(B) not numerically positive definite         */
    M2N_ERR_NO_CONVERGE = -4,  /* eigen-solver did not reach its tolerance       */
    M2N_ERR_OOM = -5,          /* device allocation or memory budget exceeded    */
    M2N_ERR_HIP = -6,          /* a HIP runtime call failed                      */
    M2N_ERR_NOT_READY = -7,    /* queue: request still in flight                 */
    M2N_ERR_UNSUPPORTED = -8,  /* valid input outside what this build implements */
    M2N_ERR_CANCELLED = -9     /* queue: request cancelled by queue destruction  */
} m2n_status;

typedef enum { M2N_FP32 = 1, M2N_FP64 = 2 } m2n_prec;

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` caps the
 * library's own workspace (0 = no cap).  On success *out owns all plans,
 * caches and workspace until m2n_destroy. */
int m2n_create(int hip_device, size_t hbm_budget_bytes, m2n_ctx **out);

/* Free everything the context owns (waits for its streams' work first). */
void m2n_destroy(m2n_ctx *ctx);

/* Text of the last failure on the calling thread ("" if none).  The text is
 * kept per thread, not per context: `ctx` is not read and may be NULL. */
const char *m2n_last_error(const m2n_ctx *ctx);

/* Bytes of device workspace the context currently holds. */
size_t m2n_workspace_bytes(const m2n_ctx *ctx);

/*
 * gpss_tapers -- Table 3 step 3, GEP branch (Sec. 3.2): the K largest
 * generalized eigenpairs of R(A0) w = lambda R(B) w at f_c0 = 0.
 *
 *   t       [N]     device, FP64, strictly increasing sampling times
 *   fmax            signal band half-width, > f_w
 *   fw              nominal band half-width, > 0
 *   fc0             nominal band centre; only 0 is implemented here (else
 *                   M2N_ERR_UNSUPPORTED); a centre fc0 != 0 gives complex
 *                   tapers: gpss_tapers_subband
 *   w       [K*N]   device, FP64 out: taper k at w + k*N, w_k^T R(B) w_k = 2 f_w;
 *                   sign: the larger in magnitude of sum_n w_k(t_n) and
 *                   sum_n (tbar - t_n) w_k(t_n) is positive, tbar = (t_1+t_N)/2
 *   lambda  [K]     device, FP64 out, descending, in [0, 1]
 *
 * The call checks t on the device (t is never copied to the host); the
 * path depends on what the check finds (t on an integer lattice or not, t_1,
 * t_N).  The first call on given t buffers (pointer and N) waits for the
 * check; the context keeps its records, and later calls on the same buffers
 * queue the tapers on them and compare them with the real check once all is
 * queued, recomputing on a difference (as m2n_batch_psd).  When R(B) is a
 * multiple of the identity (t on an integer lattice, 2 f_max a positive
 * integer) the tapers are stream-ordered and the call returns before they
 * are complete; otherwise (dense R(B), or the subspace-iteration fallback
 * for wide bands) it blocks until they are, since it reads back the
 * Cholesky or convergence status.  Errors: M2N_ERR_ARG (non-finite t), M2N_ERR_T_ORDER,
 * M2N_ERR_NOT_PD (Cholesky pivot <= 0; no silent regularisation),
 * M2N_ERR_NO_CONVERGE, M2N_ERR_UNSUPPORTED (dense N > 65536).
 */
int gpss_tapers(m2n_ctx *ctx, void *stream, const double *t, int64_t N,
                double fmax, double fw, double fc0, int K,
                double *w, double *lambda);

/*
 * gpss_tapers_rr -- gpss_tapers when R(B) may be numerically singular (the
 * GEP of Sec. 3.2 assumes it positive definite): a rank-revealing reduction.
 * A diagonally pivoted Cholesky of R(B) takes, one at a time, the sample
 * with the largest remaining Schur diagonal (ties within 1e-12 relative to
 * the smallest index) until every remaining one is below rank_tol * 2 f_max;
 * the tapers are those of gpss_tapers on the kept samples t_S (increasing
 * order; sign reading on t_S) and are zero on the others, so that
 * w_k^T R(B) w_k = 2 f_w with the full R(B).  When R(B) is a multiple of the
 * identity (integer t, integer 2 f_max) every sample is kept.
 *
 *   t, N, fmax, fw, K, w, lambda   as in gpss_tapers (fc0 = 0)
 *   rank_tol        relative pivot floor in (0, 1); <= 0: 1e-8.  The GEP of
 *                   t_S then has cond(R(B)_SS) of order 1 / rank_tol, which
 *                   bounds its forward error
 *   rank    [1]     HOST out: the number of samples kept
 *
 * Blocks (the pivot steps read a stop flag every 16 steps).  N <= 32768.
 * Errors: as gpss_tapers; M2N_ERR_NOT_PD when fewer than K samples are kept.
 */
int gpss_tapers_rr(m2n_ctx *ctx, void *stream, const double *t, int64_t N,
                   double fmax, double fw, int K, double rank_tol,
                   double *w, double *lambda, int64_t *rank);

/*
 * m2nufft_psd_at -- Table 3 steps 4 and 5 at an arbitrary list of band
 * centres (Sec. 3.2; the centres need not be equally spaced), by direct FP64
 * summation: J_k(i) = sum_n w_k(t_n) x(t_n) e^{-j 2 pi f_i t_n} and
 * P_i = sum_k d_k |J_k(i)|^2.  Costs N*I complex exponentials: meant for a
 * modest number of centres (for many equally spaced ones use m2nufft_psd).
 *
 *   t, x    [N]     device, FP64
 *   w       [K*N]   device, FP64 real tapers, 1 <= K <= 64 (summed in groups
 *                   of 16 tapers)
 *   freqs   [I]     device, FP64 band centres, any order, repeats allowed
 *   weights [K]     device, FP64 d_k, or NULL for d_k = 1/K
 *   P       [I]     device out, FP64
 *   J       [K*I]   device out or NULL, double2
 *
 * Stream-ordered and asynchronous.  Errors: M2N_ERR_ARG.
 */
int m2nufft_psd_at(m2n_ctx *ctx, void *stream, const double *t, const double *x,
                   int64_t N, const double *w, int K, const double *freqs,
                   int64_t I, const double *weights, double *P, void *J);

/*
 * m2nufft_psd_freqs -- the same quantities at an arbitrary list of band
 * centres by a type-3 NuFFT, for many centres: with t_c an integer centre of
 * the span and X the half-span, the samples are divided by the Fourier
 * transform of an exponential-of-semicircle kernel psi of w cells of a
 * frequency grid of spacing d = 1/(4 X), the library's type-1 NuFFT puts
 * them on the grid covering [min f_i, max f_i] (about 4 X (max f_i - min f_i)
 * bands), and each centre interpolates w grid values with psi (FP64) and
 * takes the phase e^{-j 2 pi f_i t_c}.  The kernel width is
 * ceil(-log10 tol) + 2 and the inner NuFFT runs a decade tighter, so J and P
 * hold tol relative to their largest values.
 *
 *   t, x    [N]     device, FP64 (any order)
 *   w       [K*N]   device, FP64 real tapers, 1 <= K <= 64
 *   freqs   [I]     device, FP64 band centres, any order, repeats allowed
 *   prec            M2N_FP32 (P float, J float2; inner NuFFT FP32) or
 *                   M2N_FP64 (double, double2)
 *   nufft_tol       requested accuracy (<= 0: 1e-6 FP32, 1e-12 FP64)
 *   weights [K]     device, FP64 d_k, or NULL for d_k = 1/K
 *   P       [I]     device out; J [K*I] device out or NULL
 *
 * One host round trip (the span of t and of the centres sizes the grid).
 * Errors: M2N_ERR_ARG, M2N_ERR_UNSUPPORTED (grid above 2^21 bands:
 * 4 X (max f_i - min f_i) too large).
 */
int m2nufft_psd_freqs(m2n_ctx *ctx, void *stream, const double *t, const double *x,
                      int64_t N, const double *w, int K, const double *freqs,
                      int64_t I, int prec, double nufft_tol, const double *weights,
                      void *P, void *J);

/*
 * m2nufft_psd_at_noalloc -- m2nufft_psd_at for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, layouts and results (the sample
 * chunks' partial sums are added in the same chunk order; when they would not
 * fit, fewer and longer chunks are used, which changes the FP64 rounding
 * only).  The partial sums live in a library-owned device array of 16 MiB
 * per GPU (M2N_NOALLOC_SCRATCH_BYTES), held from m2n_create until the
 * process ends; the call allocates nothing, grows no workspace and records no
 * timing events.
 *
 * Limits and sharing: min(K, 16) * I * 16 bytes must not exceed the array
 * (I <= 65536 for any K), else M2N_ERR_ARG.  Every call on one GPU uses the same
 * array: calls that overlap on one GPU (different streams, threads or
 * contexts without ordering between them) race and give wrong results.
 * Stream-ordered and asynchronous.  Errors: M2N_ERR_ARG.
 */
#define M2N_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int m2nufft_psd_at_noalloc(m2n_ctx *ctx, void *stream, const double *t,
                           const double *x, int64_t N, const double *w, int K,
                           const double *freqs, int64_t I,
                           const double *weights, double *P, void *J);

/*
 * idpss_tapers -- the interpolated-DPSS branch of Table 3 step 3 (nominal band
 * centred at 0; Table 3 in Sec. 3.7): tapers that approximate the GPSS tapers without a
 * GEP on t.
 *   (a) the DPSS of length N and half-bandwidth f_w D on the uniform grid
 *       t_1 + m D, D = (t_N - t_1) / (N - 1);
 *   (b) the natural cubic spline through those values, evaluated at t_n;
 *   (c) the scale w_k^T R(B) w_k = 2 f_w (R(B) of the band |f| <= f_max);
 *       sign as in gpss_tapers.
 *
 *   t       [N]     device, FP64, strictly increasing, N >= 2
 *   fmax, fw        0 < fw < fmax; f_w D < 1/2
 *   K               1 <= K <= min(N, 32)
 *   w       [K*N]   device, FP64 out, taper k at w + k*N
 *   lambda  [K]     device, FP64 out: the concentrations of the uniform-grid
 *                   DPSS, descending (the interpolated tapers solve no GEP)
 *
 * The scale costs O(N) when R(B) is a multiple of the identity (every t_n an
 * integer and 2 f_max a positive integer), else an O(N^2) FP64 quadratic
 * form.  The call waits for its check of t (one round trip) and for the DPSS
 * solve's; the rest is stream-ordered.  Errors: M2N_ERR_ARG (bad sizes or
 * bands, non-finite t), M2N_ERR_T_ORDER.
 */
int idpss_tapers(m2n_ctx *ctx, void *stream, const double *t, int64_t N,
                 double fmax, double fw, int K, double *w, double *lambda);

/*
 * gpss_tapers_subband -- one sub-band of the multiband partition (Sec. 2.4
 * sub-band matrix, Appendix A; Sec. 3.1 nominal band; Sec. 3.2 GEP at A0):
 * the K largest solutions of R(A0) w = lambda R(B^q) w, where B^q is
 * f_min <= |f| <= f_max with R(B^q)(tau) = 2 cos(pi (f_max + f_min) tau)
 * sin(pi (f_max - f_min) tau) / (pi tau), and A0 is |f - fc0| <= f_w with the
 * complex Hermitian R(A0)(tau) = e^{j 2 pi fc0 tau} sin(2 pi f_w tau) / (pi tau).
 * The tapers are complex.
 *
 *   t       [N]     device, FP64, strictly increasing sampling times
 *   fmin, fmax      sub-band edges, 0 <= fmin < fmax
 *   fw, fc0         nominal band; it must lie inside the sub-band:
 *                   |fc0| + fw <= fmax and, when fmin > 0, |fc0| - fw >= fmin
 *   K               1 <= K <= min(N, 32)
 *   w       [2*K*N] device, FP64 out, planar complex: Re w_k at w + k*N,
 *                   Im w_k at w + (K + k)*N; w_k^* R(B^q) w_k = 2 f_w; phase:
 *                   with v_n = w_k(t_n) e^{-j 2 pi fc0 (t_n - tbar)},
 *                   a = sum v_n and b = sum (tbar - t_n) v_n / (t_N - t_1),
 *                   the one of larger modulus is real and positive
 *                   (tbar = (t_1 + t_N)/2; for fc0 = 0 and real tapers this is
 *                   the sign rule of gpss_tapers)
 *   lambda  [K]     device, FP64 out, descending
 *
 * R(B^q) is always factored densely (N <= 65536).  It is positive definite
 * in exact arithmetic, but numerically singular when the sampling is denser
 * than the sub-band's Landau rate 2 (f_max - f_min) over much of the span:
 * then the Cholesky fails with M2N_ERR_NOT_PD (no silent regularisation).
 * R(A0) enters through its quadrature factor of complex rank Q =
 * ceil(0.7 * 2 pi f_w (t_N - t_1)) + 14 (even), limited to Q <= 32, i.e.
 * f_w (t_N - t_1) <= 4 (else M2N_ERR_UNSUPPORTED).  Blocks until the tapers
 * are complete.  Errors: M2N_ERR_ARG, M2N_ERR_T_ORDER, M2N_ERR_NOT_PD,
 * M2N_ERR_UNSUPPORTED.
 */
int gpss_tapers_subband(m2n_ctx *ctx, void *stream, const double *t, int64_t N,
                        double fmin, double fmax, double fw, double fc0, int K,
                        double *w, double *lambda);

/*
 * gpss_tapers_multiband -- gpss_tapers_subband for Q sub-bands at once (the
 * multiband partition of Sec. 3.1; the sub-bands are independent).  Each
 * sub-band runs on a child context of ctx (own workspace, streams and pinned
 * records, created on first use with ctx's device and memory budget, released
 * by m2n_destroy(ctx)) and a stream of its own, from a host thread of its
 * own, so that the dense factorisations of different sub-bands overlap on the
 * GPU.  Results equal the one-sub-band calls bitwise.
 *
 *   t       [N]     device, FP64 (ready on `stream`: the sub-bands wait for it)
 *   fw, K           as in gpss_tapers_subband (shared by all sub-bands)
 *   sb      [Q]     HOST array: f_min, f_max, fc0 and the device outputs w
 *                   [2*K*N] (planar complex) and lambda [K] of each sub-band
 *   Q               1 <= Q <= 16
 *
 * Blocks until every sub-band is complete.  Errors as gpss_tapers_subband;
 * the message names the first failing sub-band.  Kernel timings of the child
 * contexts are not reported by m2n_profile_read(ctx).
 */
typedef struct {
    double fmin, fmax, fc0;
    double *w, *lambda;
} m2n_subband;

int gpss_tapers_multiband(m2n_ctx *ctx, void *stream, const double *t, int64_t N,
                          double fw, int K, const m2n_subband *sb, int Q);

/*
 * m2nufft_psd_subband -- Table 3 steps 4 and 5 for one sub-band (Sec. 3.2:
 * eigencoefficients of the shifted tapers on frequencies relative to fc0):
 *   J_k(i) = sum_n conj(w_k(t_n)) x(t_n) e^{-j 2 pi (f_lo + i df) t_n},
 *   P_i    = sum_k d_k |J_k(i)|^2,
 * where f_lo + i df is the offset of band i's centre from fc0.
 *
 *   t, x    [N]     device, FP64
 *   w       [2*K*N] device, FP64 planar complex tapers (gpss_tapers_subband)
 *   K               1 <= K <= 32
 *   f_lo, df, I, prec, nufft_tol   as in m2nufft_eigcoeffs
 *   weights [K]     device, FP64 d_k, or NULL for d_k = 1/K
 *   P       [I]     device out, float (FP32) or double (FP64)
 *   J       [K*I]   device out or NULL, complex (float2 / double2)
 *
 * The 2K real and imaginary parts go through the NuFFT as 2K real tapers
 * (context workspace 2*K*I complex values), then one kernel forms J and P.
 * Stream-ordered and asynchronous once the NuFFT plan exists.
 */
int m2nufft_psd_subband(m2n_ctx *ctx, void *stream, const double *t,
                        const double *x, int64_t N, const double *w, int K,
                        double f_lo, double df, int64_t I, int prec,
                        double nufft_tol, const double *weights, void *P,
                        void *J);

/*
 * m2nufft_eigcoeffs -- Table 3 step 4 (Sec. 3.2 eigencoefficients) as a
 * type-1 NuFFT of the K tapered sequences onto the I band centres.
 *
 *   t, x    [N]     device, FP64; t strictly increasing
 *   w       [K*N]   device, FP64 tapers (any real tapers, e.g. from gpss_tapers)
 *   f_lo, df        band centres f_lo + i*df, i = 0..I-1 (df > 0)
 *   prec            M2N_FP32: spread/FFT/average in FP32 (J is float2);
 *                   M2N_FP64: all FP64 (J is double2)
 *   nufft_tol       requested relative accuracy of the NuFFT (<= 0: 1e-6 for
 *                   FP32, 1e-12 for FP64); sets the kernel width
 *   J       [K*I]   device out, complex, J + (k*I + i)
 *
 * Stream-ordered and asynchronous once the plan for (I, prec, tol) exists
 * (the first call for a plan allocates and fills its tables).
 */
int m2nufft_eigcoeffs(m2n_ctx *ctx, void *stream, const double *t,
                      const double *x, int64_t N, const double *w, int K,
                      double f_lo, double df, int64_t I, int prec,
                      double nufft_tol, void *J);

/*
 * m2nufft_psd -- Table 3 steps 4 and 5 fused, plus the suboptimality
 * estimate of Appendix B.
 *
 *   t, x, w, f_lo, df, I, prec, nufft_tol   as in m2nufft_eigcoeffs
 *   lambda  [K]     device, FP64 eigenvalues of the tapers (needed for E)
 *   fmax, fw        band parameters the tapers were built for (needed for E)
 *   weights [K]     device, FP64 d_k, or NULL for d_k = 1/K
 *   P       [I]     device out, float (FP32) or double (FP64)
 *   E       [I]     device out or NULL: Ehat_i for any strictly increasing
 *                   t.  Where R(B) is a multiple of the identity (every t_n an
 *                   integer, 2 f_max a positive integer) D_k(i) = 2 f_max
 *                   |w_k|^2 for every band and the NuFFT pass writes it.
 *                   Elsewhere D_k(i) is the integral of the taper's spectral
 *                   window |W_k(f)|^2, W_k(f) = sum_n w_k(t_n) e^{-j 2 pi f t_n},
 *                   over [f_i - f_max, f_i + f_max] (equal to the quadratic
 *                   form): Gauss-Legendre sums over cells of width df, the
 *                   window samples from batched NuFFTs of the bare tapers on
 *                   I + floor(2 f_max / df) - 1 band centres per node (work
 *                   space about (nodes * K * (I + 2 f_max / df)) reals; the
 *                   node count grows with df (t_N - t_1)).  Needs
 *                   I + 2 f_max / df <= 2^21 + 1 and df (t_N - t_1) <= about
 *                   20 there (else M2N_ERR_UNSUPPORTED), and t strictly
 *                   increasing (else M2N_ERR_T_ORDER).  The call launches a
 *                   check of t first and reads it once the NuFFT is queued
 *                   (the host waits for the check, the device does not wait
 *                   for the host).
 *   J       [K*I]   device out or NULL, as in m2nufft_eigcoeffs
 *   F       [I]     device out or NULL (same type as P): the Thomson
 *                   F-statistic of every band (Sec. 3.6), with the tapers'
 *                   DC gains W_k(0) = sum_n w_k(t_n) and C_i = sum_k J_k(i)
 *                   W_k(0) / sum_k W_k(0)^2:
 *                     F_i = |C_i|^2 (K-1) sum_k W_k(0)^2
 *                           / sum_k |J_k(i) - C_i W_k(0)|^2,
 *                   F(2, 2K-2) distributed for noise; needs K >= 2
 *                   (M2N_ERR_ARG otherwise).  +inf where the residual
 *                   vanishes.
 *
 * Stream-ordered and asynchronous once the plan exists (with E, the call
 * returns after the device has passed the check of t).
 */
int m2nufft_psd(m2n_ctx *ctx, void *stream, const double *t, const double *x,
                int64_t N, const double *w, const double *lambda, int K,
                double fmax, double fw, double f_lo, double df, int64_t I,
                int prec, double nufft_tol, const double *weights, void *P,
                void *E, void *J, void *F);

/*
 * m2n_batch_psd -- gpss_tapers followed by m2nufft_psd for many series, in
 * batched launches: one check of all sampling times, the tapers of every
 * series whose R(B) is a multiple of the identity in one set of launches
 * (the others one by one), then one NuFFT launch set per distinct band count
 * I.  Results equal the per-series calls within the NuFFT tolerance (the
 * tapers are bitwise equal).
 *
 * Host round trip: the taper path of a series depends on what the check
 * finds (t integer or not, t_1, t_N).  The first call on given t buffers
 * (pointer and N) waits for the check while the NuFFT binning runs; the
 * context keeps the records, and later calls on the same buffers queue
 * everything on them at once and compare them with the real check when all
 * is queued (by then it has long finished).  If they differ (the contents
 * changed t_1, t_N or the lattice property) the call computes everything
 * again with the real records before it returns, so results are always
 * those of the real check; an invalid t is reported as always.  Output
 * buffers hold unspecified values when a call returns an error.
 *
 *   series  [nseries] HOST array of descriptors; every pointer inside is a
 *           device pointer with the layout of the per-series calls:
 *             t, x [N]; w [K*N] out; lambda [K] out; weights [K] or NULL;
 *             P [I] out; E [I] out or NULL; J [K*I] out or NULL;
 *             F [I] out or NULL (the F-statistic, as in m2nufft_psd)
 *   prec, nufft_tol as in m2nufft_psd (one value for the whole batch)
 *
 * Errors name the offending series in m2n_last_error().  Stream-ordered
 * after the t check, except for series that take the dense or wide-band
 * taper path (see gpss_tapers), which block.  Calls on one context must not
 * run concurrently (as for every entry point).
 */
typedef struct {
    const double *t, *x;
    int64_t N;
    int K;
    double fmax, fw;
    double f_lo, df;
    int64_t I;
    const double *weights;
    double *w, *lambda;
    void *P, *E, *J;
    void *F;
} m2n_series;

int m2n_batch_psd(m2n_ctx *ctx, void *stream, const m2n_series *series, int nseries,
                  int prec, double nufft_tol);

/*
 * Replayable batches -- m2n_batch_psd for the same series launched many
 * times (fixed batch shapes: the same t, new x between launches is fine),
 * prepared once:
 *   m2n_batch_create  checks every series' t (one host round trip; each must
 *                     take the lattice path: integer t, integer 2 f_max and
 *                     quadrature rank Q + 2 <= 64, else M2N_ERR_UNSUPPORTED
 *                     naming the series), creates a child context of ctx that
 *                     owns every workspace, plan and staging block of the
 *                     batch, and runs one warm-up pass (results written).
 *                     With M2N_BATCH_TUNE it first times every NuFFT schedule
 *                     this build has kernels for at each band count of the
 *                     batch (column FFT length, pass-1 column block, pass-2
 *                     rows per workgroup; HIP events, median of three) and
 *                     keeps the fastest; the choice is appended to a text
 *                     file ($M2N_TUNE_CACHE, else
 *                     ${XDG_CACHE_HOME:-$HOME/.cache}/m2n/nufft_schedules.txt;
 *                     M2N_TUNE_CACHE="" disables it) keyed by device, band
 *                     count, precision, kernel width and the batch's size
 *                     class, and read back by later batches of that class.
 *                     With M2N_BATCH_GRAPH one more pass is captured into a
 *                     HIP graph (private capture stream).
 *   m2n_batch_launch  recomputes tapers, lambda, P, Ehat (and J, F when
 *                     given) of every series from the current contents of the
 *                     inputs: one hipGraphLaunch on `stream` with a graph,
 *                     else the same launches one by one.  No host round trip,
 *                     no allocation.  Launches on one batch must be ordered.
 *   m2n_batch_destroy waits for the device and frees the batch.
 * The series array and the device buffers it points to must outlive the
 * batch; results equal m2n_batch_psd's (tapers bitwise; P, Ehat within the
 * NuFFT tolerance when the autotuner chose another schedule).
 */
#define M2N_BATCH_GRAPH 1
#define M2N_BATCH_TUNE 2
typedef struct m2n_batch m2n_batch;
typedef struct {
    int graph;               /* 1 when launches replay a HIP graph           */
    int graph_nodes;         /* nodes of that graph                           */
    int tuned;               /* 1 when the autotuner ran                      */
    int from_cache;          /* 1 when a schedule came from the file          */
    int candidates;          /* schedules timed                               */
    int l1, B, M;            /* schedule kept for the last band count
                                (log2 N1, pass-1 block, pass-2 rows; 0 = the
                                default rule)                                  */
    double nufft_ms_default; /* NuFFT time of the default schedule (summed
                                over band counts; 0 when from the file)       */
    double nufft_ms_tuned;   /* the same for the kept schedules               */
    int series, band_counts;
} m2n_batch_info;

int m2n_batch_create(m2n_ctx *ctx, void *stream, const m2n_series *series, int nseries,
                     int prec, double nufft_tol, int flags, m2n_batch **out);
int m2n_batch_launch(m2n_batch *batch, void *stream);
int m2n_batch_get_info(const m2n_batch *batch, m2n_batch_info *info);
int m2n_batch_destroy(m2n_batch *batch);

/*
 * Request queue with continuous batching (the served form).
 *
 * Requests carry HOST inputs, which m2n_submit copies before it returns
 * (unless the queue borrows them, below), and HOST output buffers, which must
 * stay valid until m2n_poll or m2n_wait has reported the request done.  `slots` worker threads, each with its own
 * context and stream, take the pending requests in arrival order -- as many
 * as max_batch and the HBM budget admit -- and run them as one batch
 * (m2n_batch_psd); while one slot's batch is on the GPU the next admits what
 * arrived meanwhile.  A result is the same alone and in any mix within the
 * NuFFT tolerance (the tapers are bitwise equal).  The queue calls are
 * thread-safe; the parent context must outlive the queue.
 */
typedef struct m2n_queue m2n_queue;

typedef struct {
    size_t hbm_budget_bytes; /* cap on the estimated device bytes of the
                                requests in flight (0 = no cap); a request
                                larger than the cap runs alone              */
    int max_batch;           /* requests per batch (0 = 128)               */
    int slots;               /* batches in flight (0 = 4, at most 4)       */
    int prec;                /* M2N_FP32 (also when 0) or M2N_FP64         */
    double nufft_tol;        /* as in m2nufft_psd                          */
    int outputs_pinned;      /* 1: every request's host outputs are pinned
                                memory (hipHostMalloc, or a torch tensor made
                                with pin_memory=True); results are copied
                                from the device straight into them, with no
                                staging block and no host memcpy.  0: any
                                host memory, through a pinned staging block */
    int inputs_borrowed;     /* 1: m2n_submit keeps the request's t and x
                                pointers instead of copying them; the caller
                                keeps both valid and unchanged until
                                m2n_poll or m2n_wait has reported the
                                request done (or m2n_queue_destroy returned).
                                0: copied at submit                         */
} m2n_queue_cfg;

typedef struct {
    const double *t, *x;     /* HOST [N], copied by m2n_submit (or borrowed) */
    int64_t N;
    int K;
    double fmax, fw;
    double f_lo, df;
    int64_t I;
    double *w, *lambda;      /* HOST outputs [K*N], [K], or NULL             */
    void *P, *E;             /* HOST outputs [I], float (FP32) or double
                                (FP64); E NULL = not computed                */
} m2n_request;

typedef struct {
    int status;              /* M2N_OK or the request's error               */
    int batch_size;          /* requests in the batch that carried it       */
    double latency_us;       /* submit to outputs written                   */
    double service_us;       /* duration of that batch                      */
} m2n_result;

int m2n_queue_create(m2n_ctx *ctx, const m2n_queue_cfg *cfg, m2n_queue **out);
/* Errors: M2N_ERR_ARG (sizes), M2N_ERR_CANCELLED (queue shutting down). */
int m2n_submit(m2n_queue *q, const m2n_request *req, uint64_t *ticket);
/* M2N_ERR_NOT_READY while in flight; otherwise the request's status, after
 * which the ticket is released (M2N_ERR_ARG for an unknown ticket). */
int m2n_poll(m2n_queue *q, uint64_t ticket, m2n_result *res);
/* As m2n_poll after waiting up to timeout_us (< 0: without limit). */
int m2n_wait(m2n_queue *q, uint64_t ticket, m2n_result *res, int64_t timeout_us);
/* Requests not yet taken by a slot are cancelled (M2N_ERR_CANCELLED); the
 * batches on the GPU complete first.  Every ticket is invalid afterwards. */
int m2n_queue_destroy(m2n_queue *q);

/* Kernel timing.  While enabled, every kernel launch of the library is
 * bracketed by a pair of HIP events recorded on the launch stream;
 * m2n_profile_read waits for them and returns, per kernel name, the total
 * milliseconds and the number of launches since the last reset.  `names`
 * receives the names separated by '\n' (at most max_entries of them, as
 * fit into names_len bytes); the return value is the number of entries or
 * a negative m2n_status. */
int m2n_profile_enable(m2n_ctx *ctx, int on);
int m2n_profile_reset(m2n_ctx *ctx);
int m2n_profile_read(m2n_ctx *ctx, char *names, size_t names_len, double *total_ms,
                     int64_t *launches, int max_entries);

/* Wait for `stream` and report the first device-side data error flagged by
 * the library's kernels since the last check (M2N_ERR_ARG for non-finite t),
 * clearing it.  The compute calls are stream-ordered and return before their
 * kernels run, so such errors surface here.  Synchronous mode -- the library
 * built with -DM2N_SYNC=1, or a context created while the environment holds
 * M2N_SYNC=1 -- makes every compute call (and m2n_batch_launch on a batch made
 * from such a context) end with this wait and return that error itself.
 * m2n_check is the same call under its earlier name. */
int m2n_stream_status(m2n_ctx *ctx, void *stream);
int m2n_check(m2n_ctx *ctx, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* M2N_H */
