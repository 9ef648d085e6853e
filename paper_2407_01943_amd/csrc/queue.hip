// Request queue with continuous batching (the served form).
//
// m2n_submit copies a request's host inputs (or, on a queue made to borrow
// them, keeps the caller's pointers) and returns a ticket at once.
// Worker threads, one per in-flight slot, each with its own context (plans,
// workspace) and stream, take the pending requests in arrival order -- as
// many as the slot's batch limit and the queue's HBM budget admit -- stage
// their inputs in one pinned block, copy it to the device, run the batched
// path (m2n_batch_psd) and copy the outputs back.  While one slot's batch is
// on the GPU the next slot admits the requests that arrived meanwhile, so
// batches overlap on the device.  m2n_poll / m2n_wait hand back the result
// and release the ticket.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "m2n_common.hpp"

namespace m2n {
namespace {

using clk = std::chrono::steady_clock;

struct Req {
    uint64_t ticket = 0;
    std::vector<double> t, x;  // copies of the inputs (empty when borrowed)
    const double* tp = nullptr;  // the inputs: the copies or the caller's
    const double* xp = nullptr;
    int64_t N = 0, I = 0;
    int K = 0;
    double fmax = 0, fw = 0, f_lo = 0, df = 0;
    int want_E = 0;
    double* w_out = nullptr;
    double* lam_out = nullptr;
    void* P_out = nullptr;
    void* E_out = nullptr;
    size_t bytes = 0;          // device footprint estimate used for admission
    clk::time_point t_submit;
    bool done = false;
    m2n_result res{};
};

// device bytes one request needs in a batch: inputs, outputs and the
// dominant workspaces (NuFFT grids, binning arrays, quadrature basis)
size_t footprint(const Req& r, int prec) {
    const size_t cs = prec == M2N_FP32 ? 8 : 16;
    int64_t nf = 64;
    while (nf < 2 * r.I) nf *= 2;
    const size_t Np = (size_t)((r.N + 63) / 64 * 64);
    return (size_t)r.N * 16 + (size_t)r.K * r.N * 8 + (size_t)r.I * cs + (size_t)r.K * nf * cs +
           (size_t)r.N * (8 + cs + 8) + Np * 66 * 8;
}

}  // namespace
}  // namespace m2n

using namespace m2n;

struct m2n_queue {
    m2n_ctx* parent = nullptr;
    m2n_queue_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> pending;
    std::unordered_map<uint64_t, Req*> live;
    uint64_t next_ticket = 1;
    bool stopping = false;
    size_t inflight_bytes = 0;
    std::vector<std::thread> workers;
};

namespace {

struct Slot {
    m2n_ctx* ctx = nullptr;
    hipStream_t st = nullptr;
    void* dev = nullptr;       // device arena for inputs and outputs
    size_t dev_bytes = 0;
    void* pin_in = nullptr;    // pinned staging
    size_t pin_in_bytes = 0;
    void* pin_out = nullptr;
    size_t pin_out_bytes = 0;
};

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

int grow_pinned(void** p, size_t* have, size_t want) {
    if (*have >= want) return M2N_OK;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *have = 0;
    M2N_HIP(hipHostMalloc(p, want, hipHostMallocDefault));
    *have = want;
    return M2N_OK;
}

// Run one batch on a slot.  Returns the batch status; per-request statuses
// are set in the requests.
//
// Device arena: the inputs (t, x per request), then the outputs by kind, each
// kind in request order -- P and E of every request, the tapers, then the
// eigenvalues packed at 8 bytes -- so that the copies back to the host merge
// wherever the callers' buffers are contiguous too (a server's pool of
// outputs: one copy per kind and batch instead of one per output and request;
// each copy costs ~10 us of fixed overhead on top of its bytes).
int run_batch(m2n_queue* q, Slot& s, std::vector<Req*>& batch) {
    const int prec = q->cfg.prec;
    const size_t rs = prec == M2N_FP32 ? 4 : 8;
    const size_t nb = batch.size();
    size_t in_bytes = 0, pe_bytes = 0, w_bytes = 0, l_bytes = 0;
    for (Req* r : batch) {
        in_bytes += 2 * al256(sizeof(double) * r->N);
        pe_bytes += (r->want_E ? 2 : 1) * al256(rs * r->I);
        w_bytes += al256(sizeof(double) * r->K * r->N);
        l_bytes += sizeof(double) * r->K;
    }
    l_bytes = al256(l_bytes);
    const size_t out_bytes = pe_bytes + w_bytes + l_bytes;
    if (s.dev_bytes < in_bytes + out_bytes) {
        if (s.dev) {
            M2N_HIP(hipStreamSynchronize(s.st));
            (void)hipFree(s.dev);
        }
        s.dev = nullptr;
        s.dev_bytes = 0;
        const size_t want = in_bytes + out_bytes + (in_bytes + out_bytes) / 4;
        hipError_t e = hipMalloc(&s.dev, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("queue: device arena of %zu bytes: %s", want, hipGetErrorString(e));
            return M2N_ERR_OOM;
        }
        s.dev_bytes = want;
    }
    M2N_TRY(grow_pinned(&s.pin_in, &s.pin_in_bytes, in_bytes));
    if (!q->cfg.outputs_pinned) M2N_TRY(grow_pinned(&s.pin_out, &s.pin_out_bytes, out_bytes));
    char* din = (char*)s.dev;
    char* dpe = din + in_bytes;
    char* dw = dpe + pe_bytes;
    char* dl = dw + w_bytes;
    char* hin = (char*)s.pin_in;
    std::vector<m2n_series> ser(nb);
    size_t oi = 0, ope = 0, ow = 0, ol = 0;
    for (size_t j = 0; j < nb; ++j) {
        Req* r = batch[j];
        m2n_series& d = ser[j];
        std::memset(&d, 0, sizeof(d));
        std::memcpy(hin + oi, r->tp, sizeof(double) * r->N);
        d.t = (const double*)(din + oi);
        oi += al256(sizeof(double) * r->N);
        std::memcpy(hin + oi, r->xp, sizeof(double) * r->N);
        d.x = (const double*)(din + oi);
        oi += al256(sizeof(double) * r->N);
        d.N = r->N;
        d.K = r->K;
        d.fmax = r->fmax;
        d.fw = r->fw;
        d.f_lo = r->f_lo;
        d.df = r->df;
        d.I = r->I;
        d.P = dpe + ope;
        ope += al256(rs * r->I);
        d.E = nullptr;
        if (r->want_E) {
            d.E = dpe + ope;
            ope += al256(rs * r->I);
        }
        d.w = (double*)(dw + ow);
        ow += al256(sizeof(double) * r->K * r->N);
        d.lambda = (double*)(dl + ol);
        ol += sizeof(double) * r->K;
    }
    M2N_HIP(hipMemcpyAsync(din, hin, in_bytes, hipMemcpyHostToDevice, s.st));
    int st = m2n_batch_psd(s.ctx, s.st, ser.data(), (int)nb, prec, q->cfg.nufft_tol);
    if (st == M2N_OK) st = m2n_check(s.ctx, s.st);
    if (st != M2N_OK) return st;
    if (q->cfg.outputs_pinned) {
        // straight into the callers' pinned buffers, runs that are contiguous
        // on both sides merged into one copy
        struct Cp {
            char* dst;
            const char* src;
            size_t n;
        };
        std::vector<Cp> cps;
        cps.reserve(4 * nb);
        auto add = [&cps](void* dst, const void* src, size_t n) {
            char* d = (char*)dst;
            const char* sp = (const char*)src;
            if (!cps.empty() && cps.back().dst + cps.back().n == d && cps.back().src + cps.back().n == sp)
                cps.back().n += n;
            else
                cps.push_back({d, sp, n});
        };
        for (size_t j = 0; j < nb; ++j) {
            Req* r = batch[j];
            if (r->P_out) add(r->P_out, ser[j].P, rs * r->I);
            if (r->want_E && r->E_out) add(r->E_out, ser[j].E, rs * r->I);
        }
        for (size_t j = 0; j < nb; ++j)
            if (batch[j]->w_out) add(batch[j]->w_out, ser[j].w, sizeof(double) * batch[j]->K * batch[j]->N);
        for (size_t j = 0; j < nb; ++j)
            if (batch[j]->lam_out) add(batch[j]->lam_out, ser[j].lambda, sizeof(double) * batch[j]->K);
        for (const Cp& c : cps) M2N_HIP(hipMemcpyAsync(c.dst, c.src, c.n, hipMemcpyDeviceToHost, s.st));
        M2N_HIP(hipStreamSynchronize(s.st));
        for (Req* r : batch) r->res.status = M2N_OK;
        return M2N_OK;
    }
    M2N_HIP(hipMemcpyAsync(s.pin_out, dpe, out_bytes, hipMemcpyDeviceToHost, s.st));
    M2N_HIP(hipStreamSynchronize(s.st));
    const char* hout = (const char*)s.pin_out;
    for (size_t j = 0; j < nb; ++j) {
        Req* r = batch[j];
        const m2n_series& d = ser[j];
        auto host = [&](const void* dev_ptr) { return hout + ((const char*)dev_ptr - dpe); };
        if (r->w_out) std::memcpy(r->w_out, host(d.w), sizeof(double) * r->K * r->N);
        if (r->lam_out) std::memcpy(r->lam_out, host(d.lambda), sizeof(double) * r->K);
        if (r->P_out) std::memcpy(r->P_out, host(d.P), rs * r->I);
        if (r->want_E && r->E_out) std::memcpy(r->E_out, host(d.E), rs * r->I);
        r->res.status = M2N_OK;
    }
    return M2N_OK;
}

void worker(m2n_queue* q, int slot_id) {
    Slot s;
    int st = m2n_create(q->parent->device, 0, &s.ctx);
    if (st == M2N_OK && hipSetDevice(q->parent->device) == hipSuccess)
        st = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking) == hipSuccess ? M2N_OK : M2N_ERR_HIP;
    (void)slot_id;
    for (;;) {
        std::vector<Req*> batch;
        size_t bytes = 0;
        {
            std::unique_lock<std::mutex> lk(q->mu);
            q->cv_work.wait(lk, [&] { return q->stopping || !q->pending.empty(); });
            if (q->stopping) break;
            // admit in arrival order within the batch limit and the budget;
            // a request larger than the whole budget runs alone
            while (!q->pending.empty() && (int)batch.size() < q->cfg.max_batch) {
                Req* r = q->pending.front();
                const bool fits = q->cfg.hbm_budget_bytes == 0 ||
                                  q->inflight_bytes + bytes + r->bytes <= q->cfg.hbm_budget_bytes;
                if (!fits && !(batch.empty() && q->inflight_bytes == 0)) break;
                batch.push_back(r);
                bytes += r->bytes;
                q->pending.pop_front();
            }
            if (batch.empty()) {
                // budget full: wait for a running batch to release memory
                q->cv_work.wait(lk, [&] { return q->stopping || q->inflight_bytes == 0; });
                continue;
            }
            q->inflight_bytes += bytes;
        }
        const auto t0 = clk::now();
        int bst = st;
        if (bst == M2N_OK) bst = run_batch(q, s, batch);
        if (bst != M2N_OK && batch.size() > 1 && st == M2N_OK) {
            // isolate the failing request(s): one by one
            for (Req* r : batch) {
                std::vector<Req*> one{r};
                const int s1 = run_batch(q, s, one);
                if (s1 != M2N_OK) r->res.status = s1;
            }
        } else if (bst != M2N_OK) {
            for (Req* r : batch) r->res.status = bst;
        }
        const auto t1 = clk::now();
        {
            std::lock_guard<std::mutex> lk(q->mu);
            q->inflight_bytes -= bytes;
            for (Req* r : batch) {
                r->res.latency_us = std::chrono::duration<double, std::micro>(t1 - r->t_submit).count();
                r->res.service_us = std::chrono::duration<double, std::micro>(t1 - t0).count();
                r->res.batch_size = (int)batch.size();
                r->done = true;
            }
        }
        q->cv_done.notify_all();
        q->cv_work.notify_all();
    }
    if (s.st) {
        (void)hipStreamSynchronize(s.st);
        (void)hipStreamDestroy(s.st);
    }
    if (s.dev) (void)hipFree(s.dev);
    if (s.pin_in) (void)hipHostFree(s.pin_in);
    if (s.pin_out) (void)hipHostFree(s.pin_out);
    if (s.ctx) m2n_destroy(s.ctx);
}

}  // namespace

extern "C" {

int m2n_queue_create(m2n_ctx* ctx, const m2n_queue_cfg* cfg, m2n_queue** out) {
    if (!ctx || !out) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    *out = nullptr;
    m2n_queue_cfg c{};
    if (cfg) c = *cfg;
    if (c.max_batch <= 0) c.max_batch = 128;
    if (c.slots <= 0) c.slots = 4;
    if (c.slots > 4) c.slots = 4;
    if (c.prec == 0) c.prec = M2N_FP32;
    if (c.prec != M2N_FP32 && c.prec != M2N_FP64) {
        set_error("prec must be M2N_FP32 or M2N_FP64");
        return M2N_ERR_ARG;
    }
    auto* q = new (std::nothrow) m2n_queue();
    if (!q) {
        set_error("host allocation failed");
        return M2N_ERR_OOM;
    }
    q->parent = ctx;
    q->cfg = c;
    for (int i = 0; i < c.slots; ++i) q->workers.emplace_back(worker, q, i);
    *out = q;
    return M2N_OK;
}

int m2n_submit(m2n_queue* q, const m2n_request* r, uint64_t* ticket) {
    if (!q || !r || !ticket || !r->t || !r->x) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    if (r->N < 1 || r->K < 1 || r->K > 64 || r->K > r->N || r->I < 1) {
        set_error("bad request sizes (N = %lld, K = %d, I = %lld)", (long long)r->N, r->K,
                  (long long)r->I);
        return M2N_ERR_ARG;
    }
    auto* q_req = new (std::nothrow) Req();
    if (!q_req) {
        set_error("host allocation failed");
        return M2N_ERR_OOM;
    }
    Req& d = *q_req;
    if (q->cfg.inputs_borrowed) {
        d.tp = r->t;
        d.xp = r->x;
    } else {
        d.t.assign(r->t, r->t + r->N);
        d.x.assign(r->x, r->x + r->N);
        d.tp = d.t.data();
        d.xp = d.x.data();
    }
    d.N = r->N;
    d.K = r->K;
    d.I = r->I;
    d.fmax = r->fmax;
    d.fw = r->fw;
    d.f_lo = r->f_lo;
    d.df = r->df;
    d.want_E = r->E != nullptr;
    d.w_out = r->w;
    d.lam_out = r->lambda;
    d.P_out = r->P;
    d.E_out = r->E;
    d.bytes = footprint(d, q->cfg.prec);
    d.res.status = M2N_ERR_NOT_READY;
    d.t_submit = clk::now();
    {
        std::lock_guard<std::mutex> lk(q->mu);
        if (q->stopping) {
            delete q_req;
            set_error("queue is shutting down");
            return M2N_ERR_CANCELLED;
        }
        d.ticket = q->next_ticket++;
        q->live[d.ticket] = q_req;
        q->pending.push_back(q_req);
        *ticket = d.ticket;
    }
    q->cv_work.notify_one();
    return M2N_OK;
}

static int take_result(m2n_queue* q, uint64_t ticket, m2n_result* res, bool* found) {
    auto it = q->live.find(ticket);
    *found = it != q->live.end();
    if (!*found) return M2N_ERR_ARG;
    Req* r = it->second;
    if (!r->done) return M2N_ERR_NOT_READY;
    if (res) *res = r->res;
    const int st = r->res.status;
    q->live.erase(it);
    delete r;
    return st;
}

int m2n_poll(m2n_queue* q, uint64_t ticket, m2n_result* res) {
    if (!q) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(q->mu);
    bool found;
    const int st = take_result(q, ticket, res, &found);
    if (!found) set_error("unknown ticket %llu", (unsigned long long)ticket);
    return st;
}

int m2n_wait(m2n_queue* q, uint64_t ticket, m2n_result* res, int64_t timeout_us) {
    if (!q) {
        set_error("NULL argument");
        return M2N_ERR_ARG;
    }
    std::unique_lock<std::mutex> lk(q->mu);
    auto ready = [&] {
        auto it = q->live.find(ticket);
        return it == q->live.end() || it->second->done;
    };
    if (timeout_us < 0) q->cv_done.wait(lk, ready);
    else q->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    bool found;
    const int st = take_result(q, ticket, res, &found);
    if (!found) set_error("unknown ticket %llu", (unsigned long long)ticket);
    return st;
}

int m2n_queue_destroy(m2n_queue* q) {
    if (!q) return M2N_OK;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->stopping = true;
        for (Req* r : q->pending) {
            r->res.status = M2N_ERR_CANCELLED;
            r->done = true;
        }
        q->pending.clear();
    }
    q->cv_work.notify_all();
    for (auto& th : q->workers) th.join();
    for (auto& kv : q->live) delete kv.second;
    q->live.clear();
    delete q;
    return M2N_OK;
}

}  // extern "C"
