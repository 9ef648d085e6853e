// C-ABI entry points, context, workspace and error state.
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>

#include "m2n_common.hpp"

namespace m2n {

static thread_local char g_err[512] = "";

// several sub-bands at once on child contexts (subband.hip)
int multiband_run(Ctx* ctx, hipStream_t st, const double* t, int64_t N, double fw, int K, const m2n_subband* sb,
                  int Q);
// eigencoefficients at a list of band centres (nudft_list.hip)
int nudft_list_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N, const double* w, int K,
                   const double* freqs, int64_t I, const double* weights, double* P, void* J);
// the same with its partial sums in the per-device scratch array (no allocation)
int nudft_list_run_noalloc(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N, const double* w,
                           int K, const double* freqs, int64_t I, const double* weights, double* P, void* J);
// device address of that array, looked up once per device (device current)
int noalloc_scratch_init(int device);
// eigencoefficients at a list of band centres by a type-3 NuFFT (nufft3.hip)
int nufft3_run(Ctx* ctx, hipStream_t st, const double* t, const double* x, int64_t N, const double* w, int K,
               const double* freqs, int64_t I, int prec, double tol, const double* weights, void* P, void* J);
// tapers after a rank-revealing reduction of R(B) (rankrev.hip)
int gep_rr(Ctx* ctx, hipStream_t st, const double* t, int64_t N, double fmax, double fw, int K, double tau,
           double* w, double* lambda, int64_t* rank);
// interpolated-DPSS tapers (idpss.hip)
int idpss_run(Ctx* ctx, hipStream_t st, const double* t, int64_t N, double fmax, double fw, int K,
              double* w, double* lambda);

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int Ctx::alloc(DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (budget && held + bytes > budget) {
        set_error("device memory budget exceeded (%zu + %zu > %zu bytes)", held, bytes, budget);
        return M2N_ERR_OOM;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? M2N_ERR_OOM : M2N_ERR_HIP;
    }
    b.p = p;
    b.bytes = bytes;
    held += bytes;
    return M2N_OK;
}

void Ctx::release(DevBuf& b) {
    if (b.p) {
        (void)hipFree(b.p);
        held -= b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

int Ctx::workspace(const char* name, size_t bytes, void** out) {
    DevBuf& b = ws[name];
    if (b.bytes < bytes) {
        if (b.p) {
            // earlier work queued on any stream may still read the old buffer
            M2N_HIP(hipDeviceSynchronize());
            release(b);
        }
        size_t want = bytes + bytes / 4;
        M2N_TRY(alloc(b, want));
    }
    *out = b.p;
    return M2N_OK;
}

int Ctx::pinned_info(size_t bytes) {
    if (hinfo_bytes >= bytes) return M2N_OK;
    // every earlier use of the record was followed by a stream synchronise
    if (hinfo) (void)hipHostFree(hinfo);
    hinfo = nullptr;
    hinfo_bytes = 0;
    M2N_HIP(hipHostMalloc(&hinfo, bytes, hipHostMallocDefault));
    hinfo_bytes = bytes;
    return M2N_OK;
}

int Ctx::pinned_erec(size_t bytes) {
    if (erec_bytes >= bytes) return M2N_OK;
    // every earlier use of the records was followed by an event synchronise
    if (erec) (void)hipHostFree(erec);
    erec = nullptr;
    erec_bytes = 0;
    M2N_HIP(hipHostMalloc(&erec, bytes, hipHostMallocDefault));
    erec_bytes = bytes;
    return M2N_OK;
}

int Ctx::stage(hipStream_t st, const void* src, size_t bytes, void* dst_dev) {
    if (stage_fixed) {
        if (stage_cursor == stage_blocks.size()) {
            void* b = nullptr;
            M2N_HIP(hipHostMalloc(&b, bytes, hipHostMallocDefault));
            stage_blocks.push_back({b, bytes});
        } else if (stage_blocks[stage_cursor].second < bytes) {
            set_error("replayed launch sequence staged more bytes than its first pass");
            return M2N_ERR_HIP;
        }
        void* b = stage_blocks[stage_cursor++].first;
        std::memcpy(b, src, bytes);
        M2N_HIP(hipMemcpyAsync(dst_dev, b, bytes, hipMemcpyHostToDevice, st));
        return M2N_OK;
    }
    if (hstage_used) M2N_HIP(hipEventSynchronize(hstage_ev));
    if (hstage_bytes < bytes) {
        if (hstage) (void)hipHostFree(hstage);
        hstage = nullptr;
        hstage_bytes = 0;
        M2N_HIP(hipHostMalloc(&hstage, bytes + bytes / 2, hipHostMallocDefault));
        hstage_bytes = bytes + bytes / 2;
    }
    if (!hstage_ev) M2N_HIP(hipEventCreateWithFlags(&hstage_ev, hipEventDisableTiming));
    std::memcpy(hstage, src, bytes);
    M2N_HIP(hipMemcpyAsync(dst_dev, hstage, bytes, hipMemcpyHostToDevice, st));
    M2N_HIP(hipEventRecord(hstage_ev, st));
    hstage_used = true;
    return M2N_OK;
}

int Ctx::aux_stream(hipStream_t* s, hipEvent_t* fork, hipEvent_t* join) {
    if (!aux) M2N_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
    if (!aux_fork) M2N_HIP(hipEventCreateWithFlags(&aux_fork, hipEventDisableTiming));
    if (!aux_join) M2N_HIP(hipEventCreateWithFlags(&aux_join, hipEventDisableTiming));
    *s = aux;
    *fork = aux_fork;
    *join = aux_join;
    return M2N_OK;
}

hipEvent_t Ctx::take_event() {
    if (!ev_pool.empty()) {
        hipEvent_t e = ev_pool.back();
        ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int Ctx::prof_flush() {
    for (auto& r : pending) {
        M2N_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        M2N_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        auto& st = prof_stats[r.name];
        st.first += ms;
        st.second += 1;
        ev_pool.push_back(r.a);
        ev_pool.push_back(r.b);
    }
    pending.clear();
    return M2N_OK;
}

}  // namespace m2n

using namespace m2n;


#ifndef M2N_SYNC
#define M2N_SYNC 0
#endif

namespace {

// The status a compute call returns: in synchronous mode (built with
// M2N_SYNC=1, or a context created while the environment has M2N_SYNC=1) the
// call waits for its stream and reports the device-side errors its kernels
// flagged; otherwise they surface at the next m2n_stream_status.
int sync_ret(m2n_ctx* ctx, void* stream, int st) {
    if (st == M2N_OK && ctx->sync) return m2n_stream_status(ctx, stream);
    return st;
}

}  // namespace

extern "C" {

const char* m2n_last_error(const m2n_ctx* ctx) {
    (void)ctx;   // the text is kept per calling thread
    return g_err;
}

int m2n_create(int hip_device, size_t hbm_budget_bytes, m2n_ctx** out) {
    if (!out) {
        set_error("out is NULL");
        return M2N_ERR_ARG;
    }
    *out = nullptr;
    int ndev = 0;
    M2N_HIP(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev) {
        set_error("device %d out of range (%d devices)", hip_device, ndev);
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(hip_device));
    auto* c = new (std::nothrow) m2n_ctx();
    if (!c) {
        set_error("host allocation failed");
        return M2N_ERR_OOM;
    }
    c->device = hip_device;
    c->budget = hbm_budget_bytes;
    const char* sync_env = std::getenv("M2N_SYNC");
    c->sync = M2N_SYNC || (sync_env && std::strcmp(sync_env, "1") == 0);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) c->cu_count = prop.multiProcessorCount;
    void* e = nullptr;
    if (hipMalloc(&e, 256) != hipSuccess) {
        delete c;
        set_error("hipMalloc of the error word failed");
        return M2N_ERR_HIP;
    }
    (void)hipMemset(e, 0, 256);
    c->dev_err = (unsigned*)e;
    const int st = noalloc_scratch_init(hip_device);
    if (st != M2N_OK) {
        (void)hipFree(e);
        delete c;
        return st;
    }
    *out = c;
    return M2N_OK;
}

void m2n_destroy(m2n_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->plans) {
        ctx->release(kv.second->tw_fft);
        ctx->release(kv.second->inv_phihat);
    }
    for (auto& kv : ctx->fft64) {
        ctx->release(kv.second->tw);
        ctx->release(kv.second->tw_lo);
        ctx->release(kv.second->tw_hi);
    }
    for (auto& kv : ctx->ws) ctx->release(kv.second);
    for (auto& kv : ctx->gl) ctx->release(kv.second);
    if (ctx->hinfo) (void)hipHostFree(ctx->hinfo);
    if (ctx->hstage) (void)hipHostFree(ctx->hstage);
    if (ctx->hstage_ev) (void)hipEventDestroy(ctx->hstage_ev);
    if (ctx->tcheck_ev) (void)hipEventDestroy(ctx->tcheck_ev);
    if (ctx->gcheck_ev) (void)hipEventDestroy(ctx->gcheck_ev);
    if (ctx->erec) (void)hipHostFree(ctx->erec);
    for (auto& b : ctx->stage_blocks) (void)hipHostFree(b.first);
    for (auto& r : ctx->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto sst : ctx->sub_streams) (void)hipStreamDestroy(sst);
    for (auto c : ctx->subs) m2n_destroy(static_cast<m2n_ctx*>(c));
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->aux_fork) (void)hipEventDestroy(ctx->aux_fork);
    if (ctx->aux_join) (void)hipEventDestroy(ctx->aux_join);
    if (ctx->side_fork) (void)hipEventDestroy(ctx->side_fork);
    if (ctx->side_join) (void)hipEventDestroy(ctx->side_join);
    if (ctx->dev_err) (void)hipFree(ctx->dev_err);
    delete ctx;
}

size_t m2n_workspace_bytes(const m2n_ctx* ctx) { return ctx ? ctx->held : 0; }

int m2n_profile_enable(m2n_ctx* ctx, int on) {
    if (!ctx) {
        set_error("ctx is NULL");
        return M2N_ERR_ARG;
    }
    if (!on) M2N_TRY(ctx->prof_flush());
    ctx->prof = on != 0;
    return M2N_OK;
}

int m2n_profile_reset(m2n_ctx* ctx) {
    if (!ctx) {
        set_error("ctx is NULL");
        return M2N_ERR_ARG;
    }
    M2N_TRY(ctx->prof_flush());
    ctx->prof_stats.clear();
    return M2N_OK;
}

int m2n_profile_read(m2n_ctx* ctx, char* names, size_t names_len, double* total_ms,
                     int64_t* launches, int max_entries) {
    if (!ctx || !names || names_len == 0) {
        set_error("bad argument");
        return M2N_ERR_ARG;
    }
    M2N_TRY(ctx->prof_flush());
    size_t used = 0;
    int n = 0;
    names[0] = 0;
    for (auto& kv : ctx->prof_stats) {
        if (n >= max_entries) break;
        const size_t L = kv.first.size();
        if (used + L + 2 > names_len) break;
        memcpy(names + used, kv.first.c_str(), L);
        used += L;
        names[used++] = '\n';
        names[used] = 0;
        if (total_ms) total_ms[n] = kv.second.first;
        if (launches) launches[n] = kv.second.second;
        ++n;
    }
    return n;
}

int m2n_check(m2n_ctx* ctx, void* stream) { return m2n_stream_status(ctx, stream); }

int m2n_stream_status(m2n_ctx* ctx, void* stream) {
    if (!ctx) {
        set_error("ctx is NULL");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    M2N_HIP(hipStreamSynchronize((hipStream_t)stream));
    unsigned v = 0;
    M2N_HIP(hipMemcpy(&v, ctx->dev_err, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (v) {
        unsigned z = 0;
        M2N_HIP(hipMemcpy(ctx->dev_err, &z, sizeof(unsigned), hipMemcpyHostToDevice));
        if (v & DEVERR_NONFINITE) {
            set_error("non-finite sampling time or sample value");
            return M2N_ERR_ARG;
        }
    }
    return M2N_OK;
}

int gpss_tapers(m2n_ctx* ctx, void* stream, const double* t, int64_t N, double fmax, double fw,
                double fc0, int K, double* w, double* lambda) {
    if (!ctx || !t || !w || !lambda) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    if (N < 1 || K < 1 || K > 64 || K > N) {
        set_error("need 1 <= K <= min(N, 64) (N = %lld, K = %d)", (long long)N, K);
        return M2N_ERR_ARG;
    }
    if (!std::isfinite(fmax) || !std::isfinite(fw) || !(fw > 0.0) || !(fw < fmax)) {
        set_error("need 0 < fw < fmax (fw = %g, fmax = %g)", fw, fmax);
        return M2N_ERR_ARG;
    }
    if (fc0 != 0.0) {
        set_error("only f_c0 = 0 is implemented");
        return M2N_ERR_UNSUPPORTED;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, gep_run(ctx, (hipStream_t)stream, t, N, fmax, fw, K, w, lambda));
}

int m2nufft_psd_at(m2n_ctx* ctx, void* stream, const double* t, const double* x, int64_t N, const double* w,
                   int K, const double* freqs, int64_t I, const double* weights, double* P, void* J) {
    if (!ctx) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, nudft_list_run(ctx, (hipStream_t)stream, t, x, N, w, K, freqs, I, weights, P, J));
}

int gpss_tapers_rr(m2n_ctx* ctx, void* stream, const double* t, int64_t N, double fmax, double fw, int K,
                   double rank_tol, double* w, double* lambda, int64_t* rank) {
    if (!ctx) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, gep_rr(ctx, (hipStream_t)stream, t, N, fmax, fw, K, rank_tol, w, lambda, rank));
}

int m2nufft_psd_freqs(m2n_ctx* ctx, void* stream, const double* t, const double* x, int64_t N, const double* w,
                      int K, const double* freqs, int64_t I, int prec, double nufft_tol, const double* weights,
                      void* P, void* J) {
    if (!ctx) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, nufft3_run(ctx, (hipStream_t)stream, t, x, N, w, K, freqs, I, prec, nufft_tol, weights, P, J));
}

int m2nufft_psd_at_noalloc(m2n_ctx* ctx, void* stream, const double* t, const double* x, int64_t N,
                           const double* w, int K, const double* freqs, int64_t I, const double* weights,
                           double* P, void* J) {
    if (!ctx) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, nudft_list_run_noalloc(ctx, (hipStream_t)stream, t, x, N, w, K, freqs, I, weights, P, J));
}

int idpss_tapers(m2n_ctx* ctx, void* stream, const double* t, int64_t N, double fmax, double fw, int K,
                 double* w, double* lambda) {
    if (!ctx || !t || !w || !lambda) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, idpss_run(ctx, (hipStream_t)stream, t, N, fmax, fw, K, w, lambda));
}

int gpss_tapers_subband(m2n_ctx* ctx, void* stream, const double* t, int64_t N, double fmin,
                        double fmax, double fw, double fc0, int K, double* w, double* lambda) {
    if (!ctx || !t || !w || !lambda) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    if (N < 1 || K < 1 || K > 32 || K > N) {
        set_error("need 1 <= K <= min(N, 32) (N = %lld, K = %d)", (long long)N, K);
        return M2N_ERR_ARG;
    }
    if (!std::isfinite(fmin) || !std::isfinite(fmax) || !std::isfinite(fw) || !std::isfinite(fc0) ||
        !(fmin >= 0.0) || !(fmin < fmax) || !(fw > 0.0)) {
        set_error("need 0 <= fmin < fmax and fw > 0 (fmin = %g, fmax = %g, fw = %g)", fmin, fmax, fw);
        return M2N_ERR_ARG;
    }
    const double ac = std::fabs(fc0);
    if (!(ac + fw <= fmax) || (fmin > 0.0 && !(ac - fw >= fmin))) {
        set_error("the nominal band |f - %g| <= %g is not inside the sub-band %g <= |f| <= %g", fc0, fw,
                  fmin, fmax);
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, gep_subband(ctx, (hipStream_t)stream, t, N, fmin, fmax, fw, fc0, K, w, lambda));
}

int gpss_tapers_multiband(m2n_ctx* ctx, void* stream, const double* t, int64_t N, double fw, int K,
                          const m2n_subband* sb, int Q) {
    if (!ctx || !t || !sb || Q < 1 || Q > 16) {
        set_error("NULL argument or Q outside 1..16");
        return M2N_ERR_ARG;
    }
    for (int q = 0; q < Q; ++q) {
        if (!sb[q].w || !sb[q].lambda) {
            set_error("sub-band %d: NULL output", q);
            return M2N_ERR_ARG;
        }
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, multiband_run(ctx, (hipStream_t)stream, t, N, fw, K, sb, Q));
}

int m2nufft_psd_subband(m2n_ctx* ctx, void* stream, const double* t, const double* x, int64_t N,
                        const double* w, int K, double f_lo, double df, int64_t I, int prec,
                        double nufft_tol, const double* weights, void* P, void* J) {
    if (!ctx || !P) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, subband_psd_run(ctx, (hipStream_t)stream, t, x, N, w, K, f_lo, df, I, prec, nufft_tol, weights, P,
                           J));
}

int m2nufft_eigcoeffs(m2n_ctx* ctx, void* stream, const double* t, const double* x, int64_t N,
                      const double* w, int K, double f_lo, double df, int64_t I, int prec,
                      double nufft_tol, void* J) {
    if (!ctx || !J) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, nufft_run(ctx, (hipStream_t)stream, t, x, N, w, K, f_lo, df, I, prec, nufft_tol,
                     nullptr, nullptr, 0.0, 0.0, nullptr, nullptr, J, nullptr));
}

int m2nufft_psd(m2n_ctx* ctx, void* stream, const double* t, const double* x, int64_t N,
                const double* w, const double* lambda, int K, double fmax, double fw,
                double f_lo, double df, int64_t I, int prec, double nufft_tol,
                const double* weights, void* P, void* E, void* J, void* F) {
    if (!ctx || !P) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    return sync_ret(ctx, stream, nufft_run(ctx, (hipStream_t)stream, t, x, N, w, K, f_lo, df, I, prec, nufft_tol,
                     weights, lambda, fmax, fw, P, E, J, F));
}

int m2n_batch_psd(m2n_ctx* ctx, void* stream, const m2n_series* series, int nseries, int prec,
                  double nufft_tol) {
    if (!ctx || !series || nseries < 1) {
        set_error("NULL argument or empty batch");
        return M2N_ERR_ARG;
    }
    std::vector<GepIn> g((size_t)nseries);
    for (int i = 0; i < nseries; ++i) {
        const m2n_series& s = series[i];
        if (!s.t || !s.x || !s.w || !s.lambda || !s.P) {
            set_error("series %d: NULL argument", i);
            return M2N_ERR_ARG;
        }
        if (s.N < 1 || s.K < 1 || s.K > 64 || s.K > s.N) {
            set_error("series %d: need 1 <= K <= min(N, 64) (N = %lld, K = %d)", i, (long long)s.N, s.K);
            return M2N_ERR_ARG;
        }
        if (!std::isfinite(s.fmax) || !std::isfinite(s.fw) || !(s.fw > 0.0) || !(s.fw < s.fmax)) {
            set_error("series %d: need 0 < fw < fmax (fw = %g, fmax = %g)", i, s.fw, s.fmax);
            return M2N_ERR_ARG;
        }
        g[i].t = s.t;
        g[i].N = s.N;
        g[i].fmax = s.fmax;
        g[i].fw = s.fw;
        g[i].K = s.K;
        g[i].w = s.w;
        g[i].lambda = s.lambda;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    // one NuFFT batch per distinct band count; Ehat is routed here from the
    // taper solve's t check (R(B) = c I or not), so the NuFFT never waits
    struct Entry {
        int idx;
        NuSeriesIn in;
    };
    std::map<int64_t, std::vector<Entry>> groups;
    for (int i = 0; i < nseries; ++i) {
        const m2n_series& s = series[i];
        NuSeriesIn n;
        n.t = s.t;
        n.x = s.x;
        n.w = s.w;
        n.lambda = s.lambda;
        n.dk = s.weights;
        n.N = s.N;
        n.K = s.K;
        n.f_lo = s.f_lo;
        n.df = s.df;
        n.fmax = s.fmax;
        n.fw = s.fw;
        n.P = s.P;
        n.E = s.E;
        n.J = s.J;
        n.F = s.F;
        n.e_diag_known = true;
        groups[s.I].push_back({i, n});
    }
    auto ins_of = [](const std::vector<Entry>& v) {
        std::vector<NuSeriesIn> r;
        r.reserve(v.size());
        for (const Entry& e : v) r.push_back(e.in);
        return r;
    };
    // The t check, then the binning of the first band count (it needs t
    // alone), both on a side stream.  When the last call on the same t buffers left its records,
    // everything is queued at once on those and the real check (done long
    // before the host looks) is compared at the end: the parameters of the
    // taper path (lattice or not, t_1, t_N) depend on nothing else, so equal
    // records mean the queued results are the right ones; otherwise they are
    // computed again with the real records.  Without them the host waits
    // for the check alone while the binning runs.
    // The check and the binning go to the context's side stream, forked
    // from `stream` (after everything queued on it before) and joined back
    // before the NuFFT's second half, so that they run beside the tapers (the
    // taper kernels read t themselves; only their launch parameters come from
    // the check).
    hipStream_t side = nullptr;
    hipEvent_t af = nullptr, aj = nullptr;
    M2N_TRY(ctx->aux_stream(&side, &af, &aj));
    if (!ctx->side_fork) M2N_HIP(hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming));
    if (!ctx->side_join) M2N_HIP(hipEventCreateWithFlags(&ctx->side_join, hipEventDisableTiming));
    M2N_HIP(hipEventRecord(ctx->side_fork, st));
    // with the records of the last check on the same t buffers, the tapers go
    // on the stream first (they need nothing from the side stream), then the
    // check and the binning beside them
    std::unique_ptr<GepCheck, void (*)(GepCheck*)> chk_own(gep_check_new(), gep_check_free);
    GepCheck* chk = chk_own.get();
    const bool guessed = gep_check_guess(ctx, chk, g.data(), nseries);
    if (guessed) M2N_TRY(gep_run_checked(ctx, st, g.data(), nseries, chk));
    M2N_HIP(hipStreamWaitEvent(side, ctx->side_fork, 0));
    M2N_TRY(gep_check_launch(ctx, side, chk, g.data(), nseries));
    std::vector<NuSeriesIn> first = ins_of(groups.begin()->second);
    NuPending* pend = nullptr;
    M2N_TRY(nufft_begin(ctx, side, groups.begin()->first, prec, nufft_tol, first.data(), (int)first.size(), &pend));
    std::unique_ptr<NuPending, void (*)(NuPending*)> pend_own(pend, nufft_pending_free);
    M2N_HIP(hipEventRecord(ctx->side_join, side));
    if (!guessed) {
        M2N_TRY(gep_check_wait(ctx, chk, g.data(), nseries));
        M2N_TRY(gep_run_checked(ctx, st, g.data(), nseries, chk));
    }
    // the NuFFT (its first band count's binning already queued) and Ehat
    auto rest = [&](bool first_pending) -> int {
        M2N_HIP(hipStreamWaitEvent(st, ctx->side_join, 0));
        for (auto it = groups.begin(); it != groups.end(); ++it) {
            const int64_t I = it->first;
            if (it == groups.begin() && first_pending) {
                M2N_TRY(nufft_finish(ctx, st, pend_own.release()));
            } else {
                std::vector<NuSeriesIn> v = ins_of(it->second);
                M2N_TRY(nufft_run_batch(ctx, st, I, prec, nufft_tol, v.data(), (int)v.size()));
            }
            // Ehat where R(B) is not a multiple of the identity (the NuFFT
            // wrote the band-constant value, which the quadrature overwrites)
            for (const Entry& e : it->second) {
                if (!e.in.E) continue;
                int flags = 0;
                double t0 = 0.0, tN = 0.0;
                gep_check_info(chk, e.idx, &flags, &t0, &tN);
                const double c = 2.0 * e.in.fmax;
                const bool diag = !(flags & 4) && c == std::rint(c) && c >= 1.0;
                if (!diag) M2N_TRY(ehat_general(ctx, st, I, prec, nufft_tol, e.in, e.in.N > 1 ? tN - t0 : 0.0));
            }
        }
        return M2N_OK;
    };
    M2N_TRY(rest(true));
    if (guessed) {
        bool same = true;
        M2N_TRY(gep_check_confirm(ctx, chk, g.data(), nseries, &same));
        if (!same) {
            // the guess was wrong: the tapers and the NuFFT again on the real
            // records
            M2N_TRY(gep_run_checked(ctx, st, g.data(), nseries, chk));
            M2N_TRY(rest(false));
        }
    }
    return sync_ret(ctx, stream, M2N_OK);
}

}  // extern "C"
