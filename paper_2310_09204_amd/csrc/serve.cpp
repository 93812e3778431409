// Serving loop: solve requests on arbitrary multiscreens arrive at any time; up to max_inflight of
// them run concurrently on the device, each on the HIP stream of its own problem.
//
//   submit  validates the mesh on the caller's thread (sector analysis gives N), rejects requests
//           whose footprint can never fit the context's HBM budget, and queues the rest.
//   worker  takes the oldest request whose geometry is not in use and whose footprint fits next to
//           everything resident (evicting idle cached geometries, least recently used first),
//           opens a running batch for that geometry and precision with every queued request on
//           it, reuses the cached assembled matrix and preconditioner or builds them, and runs a
//           block PCG on column slots (continuous batching): requests on the same geometry that
//           arrive while the batch is assembling or solving join it and start in the slots that
//           finished columns free up; each request completes as soon as its own columns have
//           stopped.  The batch ends when no column runs and nothing waits.
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
constexpr int kSlots = 16;   // column slots of a serving batch (the block product's column group)

struct Request {
    uint64_t ticket = 0, key = 0;
    std::vector<double> V, cV, g;
    std::vector<int32_t> T, patch, cT, parent;
    int k = 0;
    bem_precision precision = BEM_FP64;
    double tol = 1e-10;
    int64_t N = 0, nt = 0;
    int64_t resident_bytes = 0, transient_bytes = 0;
    Clock::time_point t_submit, t_start, t_done;
    bool done = false;
    int rc = BEM_OK;
    std::string err;              // message of a failed request, handed to the polling thread
    std::vector<double> phi;
    std::vector<bem_solve_info> info;
    int remaining = 0;            // columns still running in a batch
    bool started = false;   // its columns entered a block PCG (t_start is set)
};

// a block PCG of one geometry and precision that takes new requests while it runs
struct Running {
    uint64_t key = 0;
    std::deque<Request*> pending;   // attached requests waiting for free column slots
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
    std::map<uint64_t, Running*> running;   // open batches by geometry key
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
        Running run;
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
                        if (r->key == pick->key) {
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
            run.key = batch[0]->key;
            run.pending.assign(batch.begin(), batch.end());
            s->running[run.key] = &run;     // later requests on this geometry attach here
        }
        // requests complete (and their polling threads free them) while the batch still runs: after
        // the solve starts, nothing here reads a request it has handed back
        Request* r0 = batch[0];
        const uint64_t key = r0->key;
        const bem_precision precision = r0->precision;
        int ktot = 0;
        for (Request* r : batch) ktot += r->k;
        const int nslots = std::max(kSlots, ktot);
        std::vector<std::pair<Request*, int>> owner(size_t(nslots), {nullptr, 0});
        int served = 0;
        Entry* entry = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            entry = &s->cache[key];
        }
        // completes r (caller holds the lock)
        auto complete = [&](Request* r, int rc, const std::string& err) {
            r->t_done = Clock::now();
            r->done = true;
            if (rc < 0) r->rc = rc;
            if (r->rc < 0) r->err = err.empty() ? "request failed" : err;
            const double lat = std::chrono::duration<double>(r->t_done - r->t_submit).count();
            const double wait = r->started ? std::chrono::duration<double>(r->t_start - r->t_submit).count() : lat;
            if (r->info.size() != size_t(r->k)) r->info.assign(size_t(r->k), bem_solve_info{});
            for (auto& in : r->info) {
                in.t_total_s = lat;
                in.t_start_s = wait;
                if (r->rc < 0 && in.status == BEM_OK && in.iters == 0) in.status = r->rc;
            }
            s->stats.completed += 1;
        };
        std::string err;
        int rc = BEM_OK;
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
            bem_problem* prob = entry->problem;
            const int64_t N = prob->N;
            HIP_CHECK(hipSetDevice(s->ctx->device));
            if (N == 0) {   // no dofs (every vertex on the boundary): the solution is empty
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->running.erase(run.key);
                    for (Request* r : run.pending) {
                        r->info.assign(size_t(r->k), bem_solve_info{});
                        complete(r, BEM_OK, "");
                    }
                    run.pending.clear();
                }
                s->cv_done.notify_all();
                throw Failure{BEM_OK, ""};
            }
            std::vector<double> col_tmp(prob->renumbered ? size_t(N) : 0);
            PcgSlots hooks;
            hooks.admit = [&](const std::vector<int>& free_slots, int running, std::vector<PcgNewColumn>& start) {
                std::lock_guard<std::mutex> lk(s->mu);
                size_t fi = 0;
                while (!run.pending.empty() && size_t(run.pending.front()->k) <= free_slots.size() - fi) {
                    Request* r = run.pending.front();
                    run.pending.pop_front();
                    r->phi.assign(size_t(N) * r->k, 0.0);
                    r->info.assign(size_t(r->k), bem_solve_info{});
                    r->remaining = r->k;
                    r->t_start = Clock::now();
                    r->started = true;
                    for (int col = 0; col < r->k; ++col) {
                        const int slot = free_slots[fi++];
                        owner[size_t(slot)] = {r, col};
                        PcgNewColumn nc{slot, {r->g[3 * col], r->g[3 * col + 1], r->g[3 * col + 2]}, r->tol};
                        start.push_back(nc);
                    }
                    if (++served == 2) s->stats.merged_batches += 1;   // counted before any request completes
                }
                if (start.empty() && running == 0) {
                    // the batch ends: requests too wide for the free slots go back to the queue front
                    s->running.erase(run.key);
                    for (auto it = run.pending.rbegin(); it != run.pending.rend(); ++it) s->queue.push_front(*it);
                    if (!run.pending.empty()) s->cv_work.notify_all();
                    run.pending.clear();
                }
            };
            hooks.finished = [&](int slot, const double* d_x, const PcgColumnResult& res) {
                auto [r, col] = owner[size_t(slot)];
                owner[size_t(slot)] = {nullptr, 0};
                if (!r) return;
                // the column in the problem's dof order, then in the caller's
                if (N > 0)
                    HIP_CHECK(hipMemcpyAsync(prob->renumbered ? col_tmp.data() : r->phi.data() + size_t(col) * N, d_x,
                                             sizeof(double) * N, hipMemcpyDeviceToHost, prob->stream));
                HIP_CHECK(hipStreamSynchronize(prob->stream));
                if (prob->renumbered)
                    for (int64_t u = 0; u < N; ++u) r->phi[size_t(col) * N + u] = col_tmp[size_t(prob->dof_int[size_t(u)])];
                bem_solve_info& in = r->info[size_t(col)];
                in.iters = res.iters;
                in.outer_iters = res.refreshes;
                in.status = res.status;
                in.graph = hooks.graphed ? 1 : 0;
                in.relres = res.relres;
                in.est_cond = std::nan("");
                if (res.status == BEM_E_BREAKDOWN) r->rc = BEM_E_BREAKDOWN;
                else if (res.status == BEM_E_NOT_CONVERGED && r->rc == BEM_OK) r->rc = BEM_E_NOT_CONVERGED;
                if (--r->remaining == 0) {
                    {
                        std::lock_guard<std::mutex> lk(s->mu);
                        complete(r, BEM_OK, res.status == BEM_E_BREAKDOWN ? "(P)CG breakdown" : "(P)CG did not converge");
                    }
                    s->cv_done.notify_all();
                }
            };
            std::lock_guard<std::mutex> call(prob->call_mu);
            (void)hipGetLastError();   // an error left by another thread's call is not this batch's
            pcg_serve(prob, entry->precond, precision == BEM_FP32_REFINE, nslots, 2000, prob->tune.check_every, hooks);
        } catch (const Failure& f) {
            rc = f.code;      // BEM_OK: the batch ended early, every request handed back
            err = f.msg;
        } catch (const std::bad_alloc&) {
            rc = BEM_E_OOM;
            err = "host allocation failed";
        } catch (const std::exception& e) {
            rc = BEM_E_DEVICE;
            err = e.what();
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (rc < 0) {
                // a failed batch fails every request it holds: running in a slot, or still waiting
                s->running.erase(run.key);
                for (auto& o : owner)
                    if (o.first && !o.first->done) {
                        Request* r = o.first;
                        for (auto& oo : owner)
                            if (oo.first == r) oo.first = nullptr;
                        complete(r, rc, err);
                    }
                for (Request* r : run.pending) complete(r, rc, err);
                run.pending.clear();
            }
            s->reserved -= reserve;
            auto it = s->cache.find(key);
            if (it != s->cache.end()) {
                it->second.busy = false;
                it->second.last_used = Clock::now();
                if (!it->second.problem) s->cache.erase(it);   // failed build
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
        auto run = s->running.find(raw->key);
        if (run != s->running.end()) {
            run->second->pending.push_back(raw);   // joins the block PCG running on its geometry
            s->stats.admitted_running += 1;
        } else {
            s->queue.push_back(raw);
            s->cv_work.notify_one();
        }
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
