// Replayable batches: the batched form (tapers and P / Ehat of many uneven
// series) prepared once and launched many times, optionally as one HIP graph,
// with the NuFFT schedule chosen by measurement.
//
//  * create: one check of every series' sampling times (each must take the
//    lattice low-rank taper path, whose launches need no host round trip),
//    a child context that owns every workspace, plan and staging block the
//    batch uses (so that captured pointers stay valid), optionally the
//    autotuner, a warm-up pass that sizes everything, and optionally the
//    capture of one more pass into a graph.
//  * launch: the graph on the caller's stream (one submission for the whole
//    batch), or the same launches issued one by one.
//  * autotuner: for every band count of the batch, the NuFFT schedules this
//    build has kernels for (column FFT length N1, pass-1 column block B,
//    pass-2 rows per workgroup M) are timed with HIP events on the batch
//    itself, the default first; the fastest is kept, and remembered in a
//    text file keyed by the device, band count, precision, kernel width and
//    the batch's size class, so that a later batch of the same class skips
//    the measurement.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <sys/stat.h>

#include "m2n_common.hpp"

namespace m2n {

namespace {

std::mutex g_tune_mu;

std::string tune_file() {
    const char* e = std::getenv("M2N_TUNE_CACHE");
    if (e) return std::string(e);   // empty: no file
    const char* xdg = std::getenv("XDG_CACHE_HOME");
    const char* home = std::getenv("HOME");
    std::string dir;
    if (xdg && *xdg) dir = std::string(xdg) + "/m2n";
    else if (home && *home) dir = std::string(home) + "/.cache/m2n";
    else return std::string();
    return dir + "/nufft_schedules.txt";
}

void make_parent_dirs(const std::string& path) {
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

int64_t pow2_at_least(int64_t v) {
    int64_t p = 1;
    while (p < v) p *= 2;
    return p;
}

bool tune_lookup(const std::string& key, NuSchedule* out) {
    const std::string f = tune_file();
    if (f.empty()) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ifstream in(f);
    if (!in) return false;
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        const size_t bar = line.find(" -> ");
        if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
        std::istringstream v(line.substr(bar + 4));
        NuSchedule s;
        if (v >> s.l1 >> s.B >> s.M) {
            *out = s;   // the last entry of a key wins
            found = true;
        }
    }
    return found;
}

void tune_store(const std::string& key, const NuSchedule& s, double ms_default, double ms_best) {
    const std::string f = tune_file();
    if (f.empty()) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    make_parent_dirs(f);
    std::ofstream out(f, std::ios::app);
    if (!out) return;
    out << key << " -> " << s.l1 << " " << s.B << " " << s.M << "   # default " << ms_default << " ms, best "
        << ms_best << " ms\n";
}

}  // namespace

}  // namespace m2n

struct m2n_batch {
    m2n_ctx* child = nullptr;
    int device = 0;
    int prec = M2N_FP32;
    double tol = 0.0;
    std::vector<m2n::GepIn> gin;
    std::vector<double> t0, tN;
    std::map<int64_t, std::vector<m2n::NuSeriesIn>> groups;   // by band count
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    m2n_batch_info info{};
};

namespace m2n {

namespace {

// every launch of one pass over the batch (no host round trip, no allocation
// once the child's workspaces have their size)
int batch_enqueue(m2n_batch* b, hipStream_t st) {
    b->child->stage_cursor = 0;
    M2N_TRY(gep_batch_enqueue_lattice(b->child, st, b->gin.data(), (int)b->gin.size(), b->t0.data(), b->tN.data()));
    for (auto& kv : b->groups)
        M2N_TRY(nufft_run_batch(b->child, st, kv.first, b->prec, b->tol, kv.second.data(), (int)kv.second.size()));
    return M2N_OK;
}

// median time of `reps` NuFFT passes over one band-count group, HIP events
int time_group(m2n_batch* b, hipStream_t st, int64_t I, std::vector<NuSeriesIn>& g, int reps, double* ms) {
    hipEvent_t e0, e1;
    M2N_HIP(hipEventCreate(&e0));
    M2N_HIP(hipEventCreate(&e1));
    std::vector<float> t;
    int rc = nufft_run_batch(b->child, st, I, b->prec, b->tol, g.data(), (int)g.size());   // builds the plan
    if (rc == M2N_OK && hipStreamSynchronize(st) != hipSuccess) rc = M2N_ERR_HIP;
    for (int r = 0; r < reps && rc == M2N_OK; ++r) {
        (void)hipEventRecord(e0, st);
        rc = nufft_run_batch(b->child, st, I, b->prec, b->tol, g.data(), (int)g.size());
        (void)hipEventRecord(e1, st);
        if (rc == M2N_OK && hipEventSynchronize(e1) != hipSuccess) rc = M2N_ERR_HIP;
        float v = 0.f;
        if (rc == M2N_OK) (void)hipEventElapsedTime(&v, e0, e1);
        t.push_back(v);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != M2N_OK) return rc;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return M2N_OK;
}

int batch_tune(m2n_batch* b, hipStream_t st) {
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) arch = prop.gcnArchName;
    for (auto& kv : b->groups) {
        const int64_t I = kv.first;
        auto& g = kv.second;
        int64_t sk = 0, sn = 0;
        for (auto& s : g) {
            sk += s.K;
            sn += s.N;
        }
        const int w = nufft_width(b->prec, b->tol);
        std::ostringstream key;
        key << arch << " I=" << I << " prec=" << b->prec << " w=" << w << " series=" << pow2_at_least((int64_t)g.size())
            << " tapers=" << pow2_at_least(sk) << " samples=" << pow2_at_least(sn);
        std::vector<NuSchedule> cand;
        M2N_TRY(nufft_schedules(I, b->prec, b->tol, cand));
        const auto pkey = std::make_tuple(I, b->prec, w);
        NuSchedule best;
        if (tune_lookup(key.str(), &best)) {
            b->info.from_cache = 1;
        } else {
            double ms_def = 0.0, ms_best = 1e300;
            for (size_t c = 0; c < cand.size(); ++c) {
                b->child->schedule[pkey] = cand[c];
                nufft_drop_plan(b->child, I, b->prec, b->tol);
                double ms = 0.0;
                const int rc = time_group(b, st, I, g, 3, &ms);
                if (rc == M2N_ERR_UNSUPPORTED) continue;   // a split this build cannot run
                M2N_TRY(rc);
                if (c == 0) ms_def = ms;
                if (ms < ms_best) {
                    ms_best = ms;
                    best = cand[c];
                }
            }
            b->info.nufft_ms_default += ms_def;
            b->info.nufft_ms_tuned += ms_best;
            b->info.candidates += (int)cand.size();
            tune_store(key.str(), best, ms_def, ms_best);
        }
        b->child->schedule[pkey] = best;
        nufft_drop_plan(b->child, I, b->prec, b->tol);
        b->info.l1 = best.l1;
        b->info.B = best.B;
        b->info.M = best.M;
    }
    b->info.tuned = 1;
    return M2N_OK;
}

void batch_free(m2n_batch* b) {
    if (!b) return;
    if (b->child) (void)hipSetDevice(b->child->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->child) m2n_destroy(b->child);
    delete b;
}

}  // namespace

}  // namespace m2n

extern "C" {

int m2n_batch_create(m2n_ctx* ctx, void* stream, const m2n_series* series, int nseries, int prec,
                     double nufft_tol, int flags, m2n_batch** out) {
    using namespace m2n;
    if (!ctx || !series || nseries < 1 || !out) {
        set_error("NULL argument or empty batch");
        return M2N_ERR_ARG;
    }
    *out = nullptr;
    if (prec != M2N_FP32 && prec != M2N_FP64) {
        set_error("prec must be M2N_FP32 or M2N_FP64");
        return M2N_ERR_ARG;
    }
    if (flags & ~(M2N_BATCH_GRAPH | M2N_BATCH_TUNE)) {
        set_error("unknown flags 0x%x", flags);
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    auto* b = new (std::nothrow) m2n_batch();
    if (!b) {
        set_error("host allocation failed");
        return M2N_ERR_OOM;
    }
    b->device = ctx->device;
    b->prec = prec;
    b->tol = nufft_tol;
    int rc = M2N_OK;
    auto fail = [&](int code) {
        batch_free(b);
        return code;
    };
    for (int i = 0; i < nseries; ++i) {
        const m2n_series& s = series[i];
        if (!s.t || !s.x || !s.w || !s.lambda || !s.P) {
            set_error("series %d: NULL argument", i);
            return fail(M2N_ERR_ARG);
        }
        if (s.N < 1 || s.K < 1 || s.K > 64 || s.K > s.N) {
            set_error("series %d: need 1 <= K <= min(N, 64) (N = %lld, K = %d)", i, (long long)s.N, s.K);
            return fail(M2N_ERR_ARG);
        }
        if (!std::isfinite(s.fmax) || !std::isfinite(s.fw) || !(s.fw > 0.0) || !(s.fw < s.fmax)) {
            set_error("series %d: need 0 < fw < fmax (fw = %g, fmax = %g)", i, s.fw, s.fmax);
            return fail(M2N_ERR_ARG);
        }
        GepIn g;
        g.t = s.t;
        g.N = s.N;
        g.fmax = s.fmax;
        g.fw = s.fw;
        g.K = s.K;
        g.w = s.w;
        g.lambda = s.lambda;
        b->gin.push_back(g);
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
        n.e_diag_known = true;   // every series is checked to be on the lattice below
        b->groups[s.I].push_back(n);
    }
    rc = m2n_create(ctx->device, ctx->budget, &b->child);
    if (rc != M2N_OK) return fail(rc);
    b->child->sync = ctx->sync;
    // the t check (one host round trip): every series on the lattice path
    rc = gep_batch_check_lattice(b->child, st, b->gin.data(), nseries, b->t0, b->tN);
    if (rc != M2N_OK) return fail(rc);
    if (flags & M2N_BATCH_TUNE) {
        // the tapers first (the NuFFT timings read them), then the schedules
        rc = gep_batch_enqueue_lattice(b->child, st, b->gin.data(), nseries, b->t0.data(), b->tN.data());
        if (rc == M2N_OK) rc = batch_tune(b, st);
        if (rc != M2N_OK) return fail(rc);
    }
    // warm-up pass: plans, workspaces and staging blocks take their sizes
    b->child->stage_fixed = true;
    rc = batch_enqueue(b, st);
    if (rc == M2N_OK && hipStreamSynchronize(st) != hipSuccess) {
        set_error("warm-up pass of the batch failed on the device");
        rc = M2N_ERR_HIP;
    }
    if (rc != M2N_OK) return fail(rc);
    if (flags & M2N_BATCH_GRAPH) {
        if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
            set_error("could not create the capture stream");
            return fail(M2N_ERR_HIP);
        }
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            set_error("hipStreamBeginCapture failed");
            return fail(M2N_ERR_HIP);
        }
        rc = batch_enqueue(b, b->cap);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->cap, &g);
        b->graph = g;
        if (rc == M2N_OK && (ec != hipSuccess || !g)) {
            set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ec));
            rc = M2N_ERR_HIP;
        }
        if (rc != M2N_OK) return fail(rc);
        const hipError_t ei = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ei));
            return fail(M2N_ERR_HIP);
        }
        size_t nn = 0;
        if (hipGraphGetNodes(b->graph, nullptr, &nn) == hipSuccess) b->info.graph_nodes = (int)nn;
        b->info.graph = 1;
    }
    b->info.series = nseries;
    b->info.band_counts = (int)b->groups.size();
    *out = b;
    return M2N_OK;
}

int m2n_batch_launch(m2n_batch* b, void* stream) {
    using namespace m2n;
    if (!b) {
        set_error("NULL batch");
        return M2N_ERR_ARG;
    }
    M2N_HIP(hipSetDevice(b->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if (b->exec) {
        M2N_HIP(hipGraphLaunch(b->exec, st));
        rc = M2N_OK;
    } else {
        rc = batch_enqueue(b, st);
    }
    // synchronous mode (as the context the batch was made from)
    if (rc == M2N_OK && b->child->sync) rc = m2n_stream_status(b->child, stream);
    return rc;
}

int m2n_batch_get_info(const m2n_batch* b, m2n_batch_info* info) {
    if (!b || !info) {
        m2n::set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    *info = b->info;
    return M2N_OK;
}

int m2n_batch_destroy(m2n_batch* b) {
    if (!b) return M2N_OK;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    m2n::batch_free(b);
    return M2N_OK;
}

}  // extern "C"
