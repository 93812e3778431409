// Serving loop: solve requests on arbitrary multiscreens arrive at any time; up to max_inflight of
// them run concurrently on the device, each on the HIP stream of its own problem.
//
//   submit  validates the mesh on the caller's thread (sector analysis gives N), rejects requests
//           whose footprint can never fit the context's HBM budget, and queues the rest.
//   worker  takes the oldest request whose geometry is not in use and whose footprint fits next to
//           everything resident (evicting idle cached geometries, least recently used first),
//           merges every queued request on the same geometry, precision and tolerance into one
//           multi-right-hand-side PCG, reuses the cached assembled matrix and preconditioner or
//           builds them, solves, and hands each request its columns.
//   poll    waits for a request and returns its result and latency (submit to completion).
//
// Footprint: resident W (8 N^2 bytes, plus 4 N^2 for the FP32 copy of mixed-precision requests)
// and the preconditioner blocks, plus, while a geometry is assembled, the pair-integral matrix
// (8 N_T^2 bytes).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <thread>

#include "internal.h"

using namespace bem;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0, key = 0;
    std::vector<double> V, cV, g;
    std::vector<int32_t> T, patch, cT, parent;
    int k = 0;
    bem_precision precision = BEM_FP64;
    double tol = 1e-10;
    int64_t N = 0, nt = 0;
    int64_t resident_bytes = 0, transient_bytes = 0;
    Clock::time_point t_submit, t_done;
    bool done = false;
    int rc = BEM_OK;
    std::string err;              // message of a failed request, handed to the polling thread
    std::vector<double> phi;
    std::vector<bem_solve_info> info;
};

struct Entry {
    bem_problem* problem = nullptr;
    bem_precond* precond = nullptr;
    int64_t bytes = 0;
    bool busy = false;
    Clock::time_point last_used;
};

uint64_t fnv(uint64_t h, const void* data, size_t n) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

struct bem_server {
    bem_ctx* ctx = nullptr;
    int max_inflight = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::map<uint64_t, Request*> requests;
    std::map<uint64_t, Entry> cache;
    std::vector<std::thread> workers;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t reserved = 0;        // bytes promised to running batches not yet in the cache
    bem_server_stats stats{};

    int64_t resident() const {
        int64_t s = 0;
        for (auto& kv : cache) s += kv.second.bytes;
        return s;
    }
};

namespace {

// evict idle cache entries (LRU) until `need` more bytes fit; caller holds the lock
bool make_room(bem_server* s, int64_t need, uint64_t keep_key) {
    const int64_t budget = int64_t(s->ctx->budget);
    while (s->resident() + s->reserved + need > budget) {
        auto victim = s->cache.end();
        for (auto it = s->cache.begin(); it != s->cache.end(); ++it) {
            if (it->second.busy || it->first == keep_key) continue;
            if (victim == s->cache.end() || it->second.last_used < victim->second.last_used) victim = it;
        }
        if (victim == s->cache.end()) return false;
        bem_precond_destroy(victim->second.precond);
        bem_problem_destroy(victim->second.problem);
        s->cache.erase(victim);
        s->stats.evictions += 1;
    }
    return true;
}

void worker_main(bem_server* s) {
    (void)hipSetDevice(s->ctx->device);
    RelaxedCapture relaxed;   // other workers capture PCG iterations concurrently
    for (;;) {
        std::vector<Request*> batch;
        bool hit = false;
        int64_t reserve = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stop) return;
                Request* pick = nullptr;
                for (Request* r : s->queue) {
                    auto it = s->cache.find(r->key);
                    if (it != s->cache.end() && it->second.busy) continue;
                    bool cached = it != s->cache.end();
                    int64_t need = cached ? 0 : r->resident_bytes + r->transient_bytes;
                    if (!make_room(s, need, r->key)) continue;
                    pick = r;
                    hit = cached;
                    reserve = need;
                    break;
                }
                if (pick) {
                    for (auto it = s->queue.begin(); it != s->queue.end();) {
                        Request* r = *it;
                        if (r->key == pick->key && r->precision == pick->precision && r->tol == pick->tol) {
                            batch.push_back(r);
                            it = s->queue.erase(it);
                        } else {
                            ++it;
                        }
                    }
                    break;
                }
                s->cv_work.wait(lk);
            }
            s->reserved += reserve;
            Entry& e = s->cache[batch[0]->key];
            e.busy = true;
            if (hit) s->stats.cache_hits += 1; else s->stats.cache_misses += 1;
            if (batch.size() > 1) s->stats.merged_batches += 1;
        }
        Request* r0 = batch[0];
        int rc = BEM_OK;
        std::string err;
        Entry* entry = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            entry = &s->cache[r0->key];
        }
        try {
            if (!entry->problem) {
                bem_assemble_opts ao{r0->precision, 10, 0, 0};
                bem_problem* p = nullptr;
                int c = bem_assemble(s->ctx, r0->V.data(), int64_t(r0->V.size() / 3), r0->T.data(), r0->nt, &ao, &p);
                if (c != BEM_OK) fail(c, bem_last_error());
                bem_precond_opts po{1, r0->precision == BEM_FP32_REFINE ? 1 : 0, 0, 0.0};
                bem_precond* m = nullptr;
                c = bem_precond_setup(p, r0->patch.data(), r0->cV.empty() ? nullptr : r0->cV.data(), int64_t(r0->cV.size() / 3),
                                      r0->cT.empty() ? nullptr : r0->cT.data(), int64_t(r0->cT.size() / 3),
                                      r0->parent.empty() ? nullptr : r0->parent.data(), &po, &m);
                if (c != BEM_OK) {
                    bem_problem_destroy(p);
                    fail(c, bem_last_error());
                }
                std::lock_guard<std::mutex> lk(s->mu);
                entry->problem = p;
                entry->precond = m;
                entry->bytes = p->bytes + m->bytes;
            }
            int ktot = 0;
            for (Request* r : batch) ktot += r->k;
            std::vector<double> g;
            for (Request* r : batch) g.insert(g.end(), r->g.begin(), r->g.end());
            bem_solve_opts o{};
            o.tol = r0->tol;
            o.max_iter = 2000;
            o.use_precond = 1;
            o.precision = r0->precision;
            o.refresh_factor = 1e-3;
            o.check_every = 4;
            o.use_graph = 1;
            const int64_t N = entry->problem->N;
            std::vector<double> phi(size_t(N) * ktot);
            std::vector<bem_solve_info> info(ktot);
            rc = bem_pcg_solve(entry->problem, entry->precond, g.data(), ktot, &o, phi.data(), info.data());
            if (rc < 0 && rc != BEM_E_NOT_CONVERGED && rc != BEM_E_BREAKDOWN) err = bem_last_error();
            int off = 0;
            for (Request* r : batch) {
                r->phi.assign(phi.begin() + size_t(off) * N, phi.begin() + size_t(off + r->k) * N);
                r->info.assign(info.begin() + off, info.begin() + off + r->k);
                int rr = BEM_OK;
                for (auto& in : r->info) {
                    if (in.status == BEM_E_BREAKDOWN) rr = BEM_E_BREAKDOWN;
                    else if (in.status == BEM_E_NOT_CONVERGED && rr == BEM_OK) rr = BEM_E_NOT_CONVERGED;
                }
                r->rc = (rc < 0 && rc != BEM_E_NOT_CONVERGED && rc != BEM_E_BREAKDOWN) ? rc : rr;
                off += r->k;
            }
        } catch (const Failure& f) {
            rc = f.code;
            err = f.msg;
            for (Request* r : batch) r->rc = rc;
        } catch (const std::bad_alloc&) {
            rc = BEM_E_OOM;
            err = "host allocation failed";
            for (Request* r : batch) r->rc = rc;
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->reserved -= reserve;
            auto it = s->cache.find(r0->key);
            if (it != s->cache.end()) {
                it->second.busy = false;
                it->second.last_used = Clock::now();
                if (!it->second.problem) s->cache.erase(it);   // failed build
            }
            const auto now = Clock::now();
            for (Request* r : batch) {
                r->t_done = now;
                r->done = true;
                if (r->rc < 0) r->err = err.empty() ? "request failed" : err;
                const double lat = std::chrono::duration<double>(r->t_done - r->t_submit).count();
                for (auto& in : r->info) in.t_total_s = lat;
                if (r->info.empty()) {
                    r->info.resize(r->k);
                    for (auto& in : r->info) { std::memset(&in, 0, sizeof(in)); in.status = r->rc; in.t_total_s = lat; }
                }
                s->stats.completed += 1;
            }
            int64_t res = s->resident();
            s->stats.resident_bytes = res;
            s->stats.peak_resident_bytes = std::max(s->stats.peak_resident_bytes, res);
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

}  // namespace

extern "C" {

int bem_server_create(bem_ctx* ctx, int max_inflight, bem_server** out) {
    try {
        if (!ctx || !out) fail(BEM_E_INVALID_ARG, "NULL argument");
        auto* s = new bem_server();
        s->ctx = ctx;
        s->max_inflight = std::max(1, std::min(max_inflight, 16));
        for (int i = 0; i < s->max_inflight; ++i) s->workers.emplace_back(worker_main, s);
        *out = s;
        return BEM_OK;
    } catch (const Failure& f) {
        set_last_error(f.msg);
        return f.code;
    }
}

void bem_server_destroy(bem_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->cache) {
        bem_precond_destroy(kv.second.precond);
        bem_problem_destroy(kv.second.problem);
    }
    for (auto& kv : s->requests) delete kv.second;
    for (Request* r : s->queue) (void)r;
    delete s;
}

int bem_serve_submit(bem_server* s, const bem_request* q, uint64_t* ticket) {
    try {
        if (!s || !q || !ticket) fail(BEM_E_INVALID_ARG, "NULL argument");
        if (!q->vertices || !q->triangles || !q->patch_of_triangle || !q->g || q->k <= 0)
            fail(BEM_E_INVALID_ARG, "incomplete request");
        std::unique_ptr<Request> r(new Request());
        r->V.assign(q->vertices, q->vertices + 3 * q->nv);
        r->T.assign(q->triangles, q->triangles + 3 * q->nt);
        r->patch.assign(q->patch_of_triangle, q->patch_of_triangle + q->nt);
        if (q->ncv > 0 && q->nct > 0) {
            if (!q->coarse_vertices || !q->coarse_triangles || !q->coarse_of_triangle) fail(BEM_E_INVALID_ARG, "coarse mesh arrays missing");
            r->cV.assign(q->coarse_vertices, q->coarse_vertices + 3 * q->ncv);
            r->cT.assign(q->coarse_triangles, q->coarse_triangles + 3 * q->nct);
            r->parent.assign(q->coarse_of_triangle, q->coarse_of_triangle + q->nt);
        }
        r->g.assign(q->g, q->g + 3 * q->k);
        r->k = q->k;
        r->precision = q->precision;
        r->tol = q->tol > 0 ? q->tol : 1e-10;
        r->nt = q->nt;
        MeshTopo m;
        analyze_mesh(q->vertices, q->nv, q->triangles, q->nt, m);
        r->N = m.N;
        const int64_t ld = ((m.N + 63) / 64) * 64;
        r->resident_bytes = ld * m.N * (r->precision == BEM_FP32_REFINE ? 12 : 8) + 2 * ld * m.N * 8 / 4;
        r->transient_bytes = q->nt * q->nt * 8;
        uint64_t h = 1469598103934665603ull;
        h = fnv(h, r->V.data(), r->V.size() * 8);
        h = fnv(h, r->T.data(), r->T.size() * 4);
        h = fnv(h, r->patch.data(), r->patch.size() * 4);
        h = fnv(h, r->cV.data(), r->cV.size() * 8);
        h = fnv(h, r->cT.data(), r->cT.size() * 4);
        h = fnv(h, r->parent.data(), r->parent.size() * 4);
        h = fnv(h, &r->precision, sizeof(r->precision));
        r->key = h;
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.submitted += 1;
        if (r->resident_bytes + r->transient_bytes > int64_t(s->ctx->budget)) {
            s->stats.rejected += 1;
            fail(BEM_E_ADMISSION, "request footprint " + std::to_string(r->resident_bytes + r->transient_bytes) +
                                      " bytes exceeds the HBM budget");
        }
        r->ticket = s->next_ticket++;
        r->t_submit = Clock::now();
        *ticket = r->ticket;
        Request* raw = r.release();
        s->requests[raw->ticket] = raw;
        s->queue.push_back(raw);
        s->cv_work.notify_one();
        return BEM_OK;
    } catch (const Failure& f) {
        set_last_error(f.msg);
        return f.code;
    }
}

int bem_serve_ndofs(bem_server* s, uint64_t ticket, int64_t* n_dofs) {
    if (!s || !n_dofs) return BEM_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) {
        set_last_error("unknown ticket");
        return BEM_E_INVALID_ARG;
    }
    *n_dofs = it->second->N;
    return BEM_OK;
}

int bem_serve_poll(bem_server* s, uint64_t ticket, int64_t timeout_us, double* phi_out, bem_solve_info* info) {
    if (!s) return BEM_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) {
        set_last_error("unknown ticket");
        return BEM_E_INVALID_ARG;
    }
    Request* r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_us < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return BEM_PENDING;
    if (phi_out && !r->phi.empty()) std::memcpy(phi_out, r->phi.data(), sizeof(double) * r->phi.size());
    if (info) std::memcpy(info, r->info.data(), sizeof(bem_solve_info) * r->info.size());
    const int rc = r->rc;
    if (rc < 0) set_last_error(r->err);
    s->requests.erase(it);
    delete r;
    return rc;
}

int bem_server_get_stats(bem_server* s, bem_server_stats* st) {
    if (!s || !st) return BEM_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->stats;
    st->resident_bytes = s->resident();
    return BEM_OK;
}

}  // extern "C"
