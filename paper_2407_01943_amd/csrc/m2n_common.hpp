// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/m2n.h"

namespace m2n {

// ---------------------------------------------------------------- complex
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R x, y;
};

template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) {
    return {a.x + b.x, a.y + b.y};
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) {
    return {a.x - b.x, a.y - b.y};
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) {
    return {a.x * s, a.y * s};
}

// ------------------------------------------------------------- error state
void set_error(const char* fmt, ...);

#define M2N_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) {                                              \
            ::m2n::set_error("%s failed: %s (%s:%d)", #call,                 \
                             hipGetErrorString(e_), __FILE__, __LINE__);     \
            return M2N_ERR_HIP;                                              \
        }                                                                    \
    } while (0)

#define M2N_TRY(expr)                 \
    do {                              \
        int s_ = (expr);              \
        if (s_ != M2N_OK) return s_;  \
    } while (0)

// Device-side sticky error bits (OR-ed by kernels, read by m2n_check).
enum : unsigned {
    DEVERR_NONFINITE = 1u,     // a non-finite t or x reached a kernel
};

// ---------------------------------------------------------- device buffers
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// --------------------------------------------------------------- NuFFT plan
struct NufftPlan {
    int64_t I = 0;     // number of bands
    int64_t h = 0;     // mode offset: band i <-> mode i - h
    int prec = 0;      // M2N_FP32 / M2N_FP64
    int w = 0;         // kernel width (cells)
    double beta = 0;   // ES kernel shape
    int nf = 0;        // fine grid size (power of two, >= 2 I)
    int log_nf = 0;
    bool single = false;   // whole grid in one workgroup's LDS
    int N1 = 0, N2 = 0;    // nf = N1 * N2 (two-pass)
    int B = 0, M = 0;      // pass-1 column block, pass-2 rows per workgroup (max)
    int KC = 0;            // pass-2 tapers transformed together
    int lookback = 0;      // extra column blocks a point may reach into
    DevBuf tw_fft;         // e^{-2 pi i j / Nt}, j < Nt (Nt = max FFT length)
    int tw_len = 0;
    DevBuf inv_phihat;     // 1 / phihat(|k|), |k| <= kmax
    int64_t kmax = 0;
    int M_force = 0;       // pass-2 rows per workgroup forced by a schedule (0: by occupancy)
};

// One series of a NuFFT launch, as the host describes it (all pointers are
// device pointers; P, E, J may be NULL as in m2nufft_psd).
struct NuSeriesIn {
    const double* t = nullptr;
    const double* x = nullptr;
    const double* w = nullptr;        // K x N tapers
    const double* lambda = nullptr;   // needed for E
    const double* dk = nullptr;       // weights or NULL (1/K)
    int64_t N = 0;
    int K = 0;
    double f_lo = 0, df = 0, fmax = 0, fw = 0;
    void* P = nullptr;
    void* E = nullptr;
    void* J = nullptr;
    void* F = nullptr;   // Thomson F-statistic [I] or NULL
    double* hrec = nullptr;   // pinned record of the t check (set internally)
    bool e_diag_known = false;  // R(B) = c I established by the caller: Ehat
                                // needs no routing (no host wait)
};

// NuFFT schedule of a plan (the autotuner's choices): log2 of the column
// FFT length N1 (0: default), pass-1 column block B (0: default), pass-2 rows
// per workgroup M (0: default)
struct NuSchedule {
    int l1 = 0, B = 0, M = 0;
};

// FP64 complex FFT plan of length M (lattice convolution in the GEP)
struct FftPlan64 {
    int64_t M = 0;
    int log_M = 0;
    bool single = false;
    int N1 = 0, N2 = 0, BB = 0, MM = 0, lo_bits = 0, tw_len = 0;
    DevBuf tw, tw_lo, tw_hi;
};

struct Ctx;

// Per-kernel timing with HIP events on the launch stream (off by default).
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};

// NuFFT entries used by the C-ABI (defined in nufft.hip)
int nufft_run(Ctx* ctx, hipStream_t st, const double* t, const double* x,
              int64_t N, const double* w, int K, double f_lo, double df,
              int64_t I, int prec, double tol, const double* weights,
              const double* lambda, double fmax, double fw, void* P, void* E,
              void* J, void* F);
// many series with one band count I and precision in one set of launches
int nufft_run_batch(Ctx* ctx, hipStream_t st, int64_t I, int prec, double tol,
                    const NuSeriesIn* series, int nseries);
// The same in two halves: nufft_begin queues the binning (it reads t
// alone), nufft_finish the rest (scatter with the tapers, both passes,
// outputs).  Ehat must be routed by the caller (e_diag_known set on every
// series with E); the NuFFT's workspace stays reserved in between, so no
// other NuFFT may run on this context until nufft_finish (or
// nufft_pending_free) is called.
struct NuPending;
int nufft_begin(Ctx* ctx, hipStream_t st, int64_t I, int prec, double tol, const NuSeriesIn* series,
                int nseries, NuPending** out);
int nufft_finish(Ctx* ctx, hipStream_t st, NuPending* pending);   // frees pending
void nufft_pending_free(NuPending* pending);
// the kernel width a tolerance gives, and every schedule this build has
// kernels for at (I, prec, width); the first entry is the default one
int nufft_width(int prec, double tol);
int nufft_schedules(int64_t I, int prec, double tol, std::vector<NuSchedule>& out);
// forget the plan of (I, prec, tol) so that the next call builds it anew
void nufft_drop_plan(Ctx* ctx, int64_t I, int prec, double tol);

// GEP entries (defined in gep.hip)
int gep_run(Ctx* ctx, hipStream_t st, const double* t_dev, int64_t N,
            double fmax, double fw, int K, double* w, double* lambda);
// one sub-band f_min <= |f| <= f_max, nominal band centre fc0: complex tapers,
// planar (real parts K x N, then imaginary parts K x N)
int gep_subband(Ctx* ctx, hipStream_t st, const double* t_dev, int64_t N, double fmin,
                double fmax, double fw, double fc0, int K, double* w, double* lambda);
// eigencoefficients and PSD of one sub-band's complex tapers (subband.hip)
int subband_psd_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N,
                    const double* w, int K, double f_lo, double df, int64_t I, int prec, double tol,
                    const double* weights, void* P, void* J);
// one series of a taper solve (device pointers; w is K x N, lambda K)
struct GepIn {
    const double* t = nullptr;
    int64_t N = 0;
    double fmax = 0, fw = 0;
    int K = 0;
    double* w = nullptr;
    double* lambda = nullptr;
};
// many series: one t check for all, the lattice low-rank ones in one set of
// launches, the rest one by one
int gep_run_batch(Ctx* ctx, hipStream_t st, const GepIn* in, int nseries);
// The same with the t check split off: gep_check_begin queues the check and
// marks its end with an event; gep_check_wait waits for that event alone
// (work queued after the check keeps running) and reads the records;
// gep_run_checked computes the tapers.  gep_check_info reports what the
// check found for series i: flags (1 non-finite, 2 not increasing, 4 some t
// not an integer), t_1 and t_N.
struct GepCheck;
int gep_check_begin(Ctx* ctx, hipStream_t st, const GepIn* in, int nseries, GepCheck** out);
// the two halves of gep_check_begin: an empty check (for gep_check_guess
// before anything is queued), then the check queued on st
GepCheck* gep_check_new();
int gep_check_launch(Ctx* ctx, hipStream_t st, GepCheck* c, const GepIn* in, int nseries);
int gep_check_wait(Ctx* ctx, GepCheck* c, const GepIn* in, int nseries);
int gep_run_checked(Ctx* ctx, hipStream_t st, const GepIn* in, int nseries, const GepCheck* c);
void gep_check_info(const GepCheck* c, int i, int* flags, double* t0, double* tN);
void gep_check_free(GepCheck* c);
// Speculation on the record of the last check of the same t buffers:
// gep_check_guess fills the records from ctx->tcache (returns false, and
// leaves them unset, unless every series has an entry that did not fail a
// guess since it last repeated); gep_check_confirm waits for the real
// check, compares, keeps the real records and reports whether they equal
// the guess (an entry that fails is not guessed on again until a waited
// check finds the same records twice in a row).  gep_check_wait also
// updates the cache.
bool gep_check_guess(Ctx* ctx, GepCheck* c, const GepIn* in, int nseries);
int gep_check_confirm(Ctx* ctx, GepCheck* c, const GepIn* in, int nseries, bool* same);
// a replayable batch: one t check, every series on the lattice low-rank path
// (gep.hip); then the tapers' launches alone
int gep_batch_check_lattice(Ctx* ctx, hipStream_t st, const GepIn* in, int ns, std::vector<double>& t0,
                            std::vector<double>& tN);
int gep_batch_enqueue_lattice(Ctx* ctx, hipStream_t st, const GepIn* in, int ns, const double* t0,
                              const double* tN);
// Ehat of one series whose R(B) is not a multiple of the identity: D_k(i) by
// quadrature of |W_k|^2 over every band's window (ehat.hip); span = t_N - t_1
int ehat_general(Ctx* ctx, hipStream_t st, int64_t I, int prec, double tol, const NuSeriesIn& s, double span);

// ----------------------------------------------------------------- context
struct Ctx {
    int device = 0;
    size_t budget = 0;         // 0 = unlimited
    size_t held = 0;           // bytes currently allocated
    std::map<std::tuple<int64_t, int, int>, std::unique_ptr<NufftPlan>> plans;
    // schedules forced for plans built from now on, by (I, prec, width)
    std::map<std::tuple<int64_t, int, int>, NuSchedule> schedule;
    // staging for replayable batches: every stage() call takes the next block
    // of its own (allocated on the first pass, reused in the same order), so
    // that a captured copy reads a block nothing else overwrites
    bool stage_fixed = false;
    std::vector<std::pair<void*, size_t>> stage_blocks;
    size_t stage_cursor = 0;
    std::map<int64_t, std::unique_ptr<FftPlan64>> fft64;   // by length
    std::map<std::string, DevBuf> ws;   // named grow-only workspaces
    unsigned* dev_err = nullptr;        // sticky device error word
    int cu_count = 256;
    bool sync = false;         // every compute call waits and reports device-side errors
    void* hinfo = nullptr;              // pinned host record of the t checks
    size_t hinfo_bytes = 0;
    std::map<int, DevBuf> gl;           // Gauss-Legendre nodes/weights by order
    // pinned staging of launch descriptors; hstage_ev marks the last copy
    // out of it, so it is rewritten only after that copy has run
    void* hstage = nullptr;
    size_t hstage_bytes = 0;
    hipEvent_t hstage_ev = nullptr;
    bool hstage_used = false;
    int stage(hipStream_t st, const void* src, size_t bytes, void* dst_dev);
    int pinned_info(size_t bytes);

    // kernel timing (m2n_profile_*)
    bool prof = false;
    std::vector<ProfRec> pending;
    std::vector<hipEvent_t> ev_pool;
    std::map<std::string, std::pair<double, int64_t>> prof_stats;   // name -> (ms, launches)
    hipEvent_t take_event();
    int prof_flush();

    // a second stream (default priority) and two events for work that
    // overlaps the caller's stream, created on first use
    hipEvent_t gcheck_ev = nullptr;     // marks the end of a taper solve's t check
    // what the last t check found per (t pointer, N): flags, t_1, t_N, and
    // whether a guess on it has failed since the records last repeated; the
    // fused call queues its tapers on these and confirms them at its end
    std::map<std::pair<const double*, int64_t>, std::tuple<int, double, double, bool>> tcache;
    hipEvent_t tcheck_ev = nullptr;     // marks the t check of an Ehat request
    void* erec = nullptr;               // pinned records of that check
    size_t erec_bytes = 0;
    int pinned_erec(size_t bytes);
    hipStream_t aux = nullptr;
    hipEvent_t aux_fork = nullptr, aux_join = nullptr;
    int aux_stream(hipStream_t* s, hipEvent_t* fork, hipEvent_t* join);
    // the fused call's fork to the side stream (t check and NuFFT binning
    // beside the tapers) and its join before the NuFFT's second half
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    // child contexts (own workspace, streams and pinned records) and their
    // streams for sub-bands solved at once; created on first use
    std::vector<Ctx*> subs;
    std::vector<hipStream_t> sub_streams;

    // grow-only named workspace; returns M2N_OK / M2N_ERR_OOM / M2N_ERR_HIP
    int workspace(const char* name, size_t bytes, void** out);
    int alloc(DevBuf& b, size_t bytes);
    void release(DevBuf& b);
};

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n)
inline void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt) {
    x.assign(n, 0.0);
    wt.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int itr = 0; itr < 100; ++itr) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(z), p0 = P_{n-1}(z)
            double dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // recompute the derivative at the converged node
                p0 = 1.0;
                p1 = z;
                for (int j = 2; j <= n; ++j) {
                    double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                x[i] = z;
                wt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
        }
    }
}

// RAII: records an event pair around the launches in its scope when timing is on
struct ProfScope {
    Ctx* c;
    hipStream_t s;
    const char* n;
    hipEvent_t a = nullptr;
    ProfScope(Ctx* c_, hipStream_t s_, const char* n_) : c(c_), s(s_), n(n_) {
        if (c && c->prof) {
            a = c->take_event();
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (a) {
            hipEvent_t b = c->take_event();
            if (b) {
                (void)hipEventRecord(b, s);
                c->pending.push_back({n, a, b});
            }
        }
    }
};

#define M2N_PROF_CAT2(a, b) a##b
#define M2N_PROF_CAT(a, b) M2N_PROF_CAT2(a, b)
#define M2N_PROF(ctx, st, name) ::m2n::ProfScope M2N_PROF_CAT(prof_scope_, __LINE__)(ctx, st, name)

}  // namespace m2n

// the opaque handle of the C-ABI is the context itself
struct m2n_ctx : public m2n::Ctx {};
