// C-ABI entry points of libbem: argument checks, handle lifetimes, error codes, host<->device copies.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>

#include "internal.h"

namespace bem {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

[[noreturn]] void fail(int code, const std::string& msg) { throw Failure{code, msg}; }

namespace {
struct Pending {
    size_t cap;
    void* ptr;
    hipEvent_t ev;
};
struct MemPool {
    std::mutex mu;
    std::multimap<size_t, void*> free;   // capacity -> buffer
    std::vector<Pending> pending;        // released, waiting for their stream
    std::vector<hipEvent_t> events;      // spare events
};
MemPool& mem_pool(int device) {
    static MemPool pools[64];
    return pools[device & 63];
}
size_t size_class(size_t b) {
    if (b >= kPooledBytes) return b;
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
}
// moves released buffers whose stream has passed the release point to the free list (lock held);
// leaves an error already pending on this thread untouched
void collect(MemPool& P) {
    if (P.pending.empty() || hipPeekAtLastError() != hipSuccess) return;
    // the events may have been recorded on a stream that another thread is now capturing, and a
    // query of such an event can invalidate that capture: while a capture is under way (it holds
    // the capture mutex) the pending buffers wait for a later allocation
    std::unique_lock<std::mutex> cap(capture_mutex(), std::try_to_lock);
    if (!cap.owns_lock()) return;
    for (size_t i = 0; i < P.pending.size();) {
        const hipError_t q = hipEventQuery(P.pending[i].ev);
        if (q == hipSuccess) {
            P.free.emplace(P.pending[i].cap, P.pending[i].ptr);
            P.events.push_back(P.pending[i].ev);
            P.pending[i] = P.pending.back();
            P.pending.pop_back();
        } else {
            (void)hipGetLastError();   // not ready: no error to keep
            ++i;
        }
    }
}
}  // namespace

std::mutex& capture_mutex() {
    static std::mutex mu;
    return mu;
}

hipStream_t acquire_stream(bem_ctx* c) {
    {
        std::lock_guard<std::mutex> lk(c->stream_mu);
        if (!c->free_streams.empty()) {
            hipStream_t st = c->free_streams.back();
            c->free_streams.pop_back();
            return st;
        }
    }
    hipStream_t st = nullptr;
    std::lock_guard<std::mutex> cap(capture_mutex());
    HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    return st;
}

void release_stream(bem_ctx* c, hipStream_t st) {
    if (!st) return;
    // a stream that is still in (or was broken by) a capture is destroyed, not handed out again:
    // every call on it would fail
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(st, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        std::lock_guard<std::mutex> cap(capture_mutex());
        (void)hipStreamDestroy(st);
        return;
    }
    std::lock_guard<std::mutex> lk(c->stream_mu);
    c->free_streams.push_back(st);
}

void release_cached_device_memory(int device) {
    MemPool& P = mem_pool(device);
    std::lock_guard<std::mutex> cap(capture_mutex());
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto& q : P.pending) {
        (void)hipEventSynchronize(q.ev);
        P.free.emplace(q.cap, q.ptr);
        P.events.push_back(q.ev);
    }
    P.pending.clear();
    for (auto& kv : P.free) (void)hipFree(kv.second);
    P.free.clear();
    for (hipEvent_t e : P.events) (void)hipEventDestroy(e);
    P.events.clear();
}

size_t available_device_bytes(int device) {
    size_t fb = 0, tb = 0;
    {
        std::lock_guard<std::mutex> cap(capture_mutex());
        HIP_CHECK(hipMemGetInfo(&fb, &tb));
    }
    MemPool& P = mem_pool(device);
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto& kv : P.free) fb += kv.first;
    for (auto& q : P.pending) fb += q.cap;
    return fb;
}

DeviceBuffer::DeviceBuffer(size_t b, hipStream_t s) : bytes(b), stream(s) {
    if (b == 0) return;
    (void)hipGetDevice(&dev);
    const size_t want = size_class(b);
    {
        MemPool& P = mem_pool(dev);
        std::lock_guard<std::mutex> lk(P.mu);
        collect(P);
        auto it = P.free.lower_bound(want);
        if (it != P.free.end() && (want < kPooledBytes ? it->first == want : it->first <= want + want / 4)) {
            ptr = it->second;
            cap = it->first;
            pooled = true;
            P.free.erase(it);
            return;
        }
    }
    // fresh allocations are rare (the pool serves repeats) and are kept apart from graph captures
    // of concurrent solves, like every other call that may synchronise the device
    auto fresh = [&]() {
        std::lock_guard<std::mutex> cap(capture_mutex());
        return hipMalloc(&ptr, want);
    };
    hipError_t e = fresh();
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        release_cached_device_memory(dev);
        e = fresh();
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
        fail(e == hipErrorOutOfMemory ? BEM_E_OOM : BEM_E_DEVICE,
             "hipMalloc(" + std::to_string(want) + " bytes): " + hipGetErrorString(e));
    }
    cap = want;
    pooled = true;
}

DeviceBuffer::~DeviceBuffer() { reset(); }

void DeviceBuffer::reset() {
    if (ptr && pooled) {
        MemPool& P = mem_pool(dev);
        std::lock_guard<std::mutex> lk(P.mu);
        hipEvent_t ev = nullptr;
        if (stream) {
            if (!P.events.empty()) {
                ev = P.events.back();
                P.events.pop_back();
            } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                ev = nullptr;
            }
            if (ev && hipEventRecord(ev, stream) != hipSuccess) {
                (void)hipGetLastError();
                P.events.push_back(ev);
                ev = nullptr;
            }
        }
        if (ev) {
            P.pending.push_back({cap, ptr, ev});
        } else if (stream) {
            // no event: wait for the stream here rather than hand out memory still in use; if
            // even that fails the buffer is not reused
            if (hipStreamSynchronize(stream) == hipSuccess) P.free.emplace(cap, ptr);
            else (void)hipGetLastError();
        } else {
            P.free.emplace(cap, ptr);
        }
    }
    ptr = nullptr;
    bytes = cap = 0;
    pooled = false;
    stream = nullptr;
}

DeviceBuffer& DeviceBuffer::operator=(DeviceBuffer&& o) noexcept {
    if (this != &o) {
        reset();
        ptr = o.ptr;
        bytes = o.bytes;
        cap = o.cap;
        dev = o.dev;
        pooled = o.pooled;
        stream = o.stream;
        o.ptr = nullptr;
        o.bytes = o.cap = 0;
        o.pooled = false;
        o.stream = nullptr;
    }
    return *this;
}

void solve_device(bem_problem* p, const bem_precond* M, const double* b, double* x, int k, const bem_solve_opts& o,
                  bem_solve_info* info);

bem_tuning tuning_for(const std::vector<bem_tuning>& table, int64_t nt) {
    bem_tuning t{};
    for (size_t i = 0; i < table.size(); ++i)
        if (nt <= table[i].max_triangles || i + 1 == table.size()) {
            t = table[i];
            break;
        }
    t.max_triangles = table.empty() ? INT64_MAX : t.max_triangles;
    if (t.far_separation <= 0) t.far_separation = 1.2;
    if (t.panel_fraction <= 0) t.panel_fraction = 0.6;
    if (t.symv_blocks_fp64 <= 0) t.symv_blocks_fp64 = 4;
    if (t.symv_blocks_fp32 <= 0) t.symv_blocks_fp32 = 8;
    if (t.check_every <= 0) t.check_every = 4;
    t.reserved = 0;
    return t;
}

}  // namespace bem

using namespace bem;

// an error left pending by calls made before this entry point belongs to those calls
#define BEM_TRY try { ::bem::RelaxedCapture relaxed_capture_guard_; (void)hipGetLastError();
#define BEM_CATCH                                              \
    }                                                          \
    catch (const Failure& f) {                                 \
        set_last_error(f.msg);                                 \
        return f.code;                                         \
    }                                                          \
    catch (const std::bad_alloc&) {                            \
        set_last_error("host out of memory");                  \
        return BEM_E_OOM;                                      \
    }                                                          \
    catch (const std::exception& e) {                          \
        set_last_error(e.what());                              \
        return BEM_E_DEVICE;                                   \
    }

namespace {

void set_device(const bem_ctx* ctx) { HIP_CHECK(hipSetDevice(ctx->device)); }

bem_solve_opts default_solve_opts() {
    bem_solve_opts o;
    std::memset(&o, 0, sizeof(o));
    o.tol = 1e-10;
    o.max_iter = 2000;
    o.use_precond = 1;
    o.precision = BEM_FP64;
    o.refresh_factor = 0.0;   // the library's default
    o.check_every = 0;   // the problem's tuned value
    o.use_graph = 1;
    return o;
}

// k columns of N values between the caller's dof order and the problem's internal one, on the
// problem's stream (src != dst)
void dofs_to_internal(const bem_problem* p, const double* src, double* dst, int k) {
    if (p->renumbered) permute_cols_device(src, p->N, dst, p->N, p->N, k, p->d_dof_user.as<int32_t>(), p->stream);
    else HIP_CHECK(hipMemcpyAsync(dst, src, sizeof(double) * p->N * k, hipMemcpyDeviceToDevice, p->stream));
}
void dofs_to_user(const bem_problem* p, const double* src, double* dst, int k) {
    if (p->renumbered) permute_cols_device(src, p->N, dst, p->N, p->N, k, p->d_dof_int.as<int32_t>(), p->stream);
    else HIP_CHECK(hipMemcpyAsync(dst, src, sizeof(double) * p->N * k, hipMemcpyDeviceToDevice, p->stream));
}
// the same on host arrays
void host_to_internal(const bem_problem* p, const double* src, double* dst, int64_t k) {
    const int64_t N = p->N;
    for (int64_t c = 0; c < k; ++c)
        for (int64_t i = 0; i < N; ++i) dst[c * N + i] = p->renumbered ? src[c * N + p->dof_user[size_t(i)]] : src[c * N + i];
}
void host_to_user(const bem_problem* p, const double* src, double* dst, int64_t k) {
    const int64_t N = p->N;
    for (int64_t c = 0; c < k; ++c)
        for (int64_t u = 0; u < N; ++u) dst[c * N + u] = p->renumbered ? src[c * N + p->dof_int[size_t(u)]] : src[c * N + u];
}

// rows of W with row and column indices in the caller's dof order, gathered on the device in
// chunks of at most 256 MB (stream-ordered behind a contraction that may still be writing W)
void copy_rows_user(const bem_problem* p, const int64_t* rows, int64_t nrows, double* out) {
    const int64_t N = p->N;
    if (N == 0 || nrows == 0) return;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nrows, (int64_t(256) << 20) / (8 * N)));
    DeviceBuffer buf(sizeof(double) * chunk * N, p->stream), drows(sizeof(int32_t) * chunk, p->stream);
    std::vector<int32_t> hr(static_cast<size_t>(chunk));
    for (int64_t r0 = 0; r0 < nrows; r0 += chunk) {
        const int64_t nr = std::min(chunk, nrows - r0);
        for (int64_t i = 0; i < nr; ++i) hr[size_t(i)] = p->dof_int[size_t(rows[r0 + i])];
        HIP_CHECK(hipMemcpyAsync(drows.ptr, hr.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice, p->stream));
        gather_rows_device(p->W64.as<double>(), p->ldw, drows.as<int32_t>(), nr, p->d_dof_int.as<int32_t>(), N,
                           buf.as<double>(), p->stream);
        HIP_CHECK(hipMemcpyAsync(out + r0 * N, buf.ptr, sizeof(double) * nr * N, hipMemcpyDeviceToHost, p->stream));
        HIP_CHECK(hipStreamSynchronize(p->stream));   // hr is refilled for the next chunk
    }
}

int solve_common(bem_problem* p, const bem_precond* m, const double* d_b, int32_t k, const bem_solve_opts* opts,
                 double* phi_out, bem_solve_info* info, double* d_phi_out = nullptr) {
    bem_solve_opts o = opts ? *opts : default_solve_opts();
    if (o.tol <= 0) o.tol = 1e-10;
    if (o.max_iter <= 0) o.max_iter = 2000;
    if (o.check_every <= 0) o.check_every = p->tune.check_every;
    if (m && m->p != p) fail(BEM_E_INVALID_ARG, "preconditioner belongs to another problem");
    const int64_t N = p->N;
    if (o.x0)
        for (int64_t i = 0; i < N * k; ++i)
            if (!std::isfinite(o.x0[i])) fail(BEM_E_INVALID_ARG, "non-finite entry in x0");
    std::vector<double> x0_int;
    if (o.x0 && p->renumbered) {
        x0_int.resize(size_t(N * k));
        host_to_internal(p, o.x0, x0_int.data(), k);
        o.x0 = x0_int.data();
    }
    std::lock_guard<std::mutex> call(p->call_mu);
    std::vector<bem_solve_info> inf(k);
    // the iterate lives in the caller's device buffer when one is given (and the problem keeps the
    // caller's order)
    DeviceBuffer x;
    const bool in_place = d_phi_out && !p->renumbered;
    if (!in_place) x = DeviceBuffer(sizeof(double) * std::max<int64_t>(1, N * k), p->stream);
    double* dx = in_place ? d_phi_out : x.as<double>();
    if (N > 0) solve_device(p, m, d_b, dx, k, o, inf.data());
    if (phi_out && !d_phi_out && N > 0) {
        std::vector<double> tmp(p->renumbered ? size_t(N * k) : 0);
        HIP_CHECK(hipMemcpyAsync(p->renumbered ? tmp.data() : phi_out, x.ptr, sizeof(double) * N * k, hipMemcpyDeviceToHost,
                                 p->stream));
        HIP_CHECK(hipStreamSynchronize(p->stream));
        if (p->renumbered) host_to_user(p, tmp.data(), phi_out, k);
    }
    if (d_phi_out && !in_place && N > 0) dofs_to_user(p, dx, d_phi_out, k);
    if (d_phi_out) HIP_CHECK(hipStreamSynchronize(p->stream));   // the caller may read it on any stream
    int rc = BEM_OK;
    for (int c = 0; c < k; ++c) {
        if (inf[c].status == BEM_E_BREAKDOWN) rc = BEM_E_BREAKDOWN;
        else if (inf[c].status == BEM_E_NOT_CONVERGED && rc == BEM_OK) rc = BEM_E_NOT_CONVERGED;
    }
    if (info) std::memcpy(info, inf.data(), sizeof(bem_solve_info) * k);
    if (rc == BEM_E_BREAKDOWN) set_last_error("(P)CG breakdown: p.Wp <= 0 or non-finite value");
    if (rc == BEM_E_NOT_CONVERGED) set_last_error("(P)CG did not reach the tolerance within max_iter");
    return rc;
}

}  // namespace

extern "C" {

const char* bem_last_error(void) { return g_last_error.c_str(); }

int bem_ctx_create(int hip_device, size_t hbm_budget_bytes, bem_ctx** out) {
    BEM_TRY
    if (!out) fail(BEM_E_INVALID_ARG, "out is NULL");
    int n = 0;
    HIP_CHECK(hipGetDeviceCount(&n));
    if (hip_device < 0 || hip_device >= n) fail(BEM_E_INVALID_ARG, "no such HIP device");
    auto* c = new bem_ctx();
    c->device = hip_device;
    HIP_CHECK(hipSetDevice(hip_device));
    size_t fr = 0, tot = 0;
    HIP_CHECK(hipMemGetInfo(&fr, &tot));
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : size_t(0.9 * double(fr));
    HIP_CHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    // this device's address of the scratch array of bem_matvec_noalloc, looked up once here
    noalloc_scratch_address(hip_device);
    *out = c;
    return BEM_OK;
    BEM_CATCH
}

int bem_ctx_set_tuning(bem_ctx* ctx, const bem_tuning* entries, int32_t n) {
    BEM_TRY
    if (!ctx || n < 0 || n > 16 || (n > 0 && !entries)) fail(BEM_E_INVALID_ARG, "bad argument");
    std::vector<bem_tuning> t(entries, entries + n);
    for (int32_t i = 0; i < n; ++i) {
        const bem_tuning& e = t[size_t(i)];
        auto bad = [&](const char* what) { fail(BEM_E_INVALID_ARG, std::string("tuning entry ") + std::to_string(i) + ": " + what); };
        if (e.max_triangles <= 0 || (i > 0 && e.max_triangles <= t[size_t(i) - 1].max_triangles)) bad("max_triangles not increasing");
        if (e.far_separation != 0 && !(e.far_separation >= 1.1 && e.far_separation <= 3.0)) bad("far_separation outside [1.1, 3]");
        if (e.panel_fraction != 0 && !(e.panel_fraction >= 0.2 && e.panel_fraction <= 0.8)) bad("panel_fraction outside [0.2, 0.8]");
        if (e.symv_blocks_fp64 != 0 && e.symv_blocks_fp64 != 2 && e.symv_blocks_fp64 != 4 && e.symv_blocks_fp64 != 8)
            bad("symv_blocks_fp64 not 2, 4 or 8");
        if (e.symv_blocks_fp32 != 0 && e.symv_blocks_fp32 != 4 && e.symv_blocks_fp32 != 8 && e.symv_blocks_fp32 != 16)
            bad("symv_blocks_fp32 not 4, 8 or 16");
        if (e.check_every < 0 || e.check_every > 64) bad("check_every outside [0, 64]");
    }
    ctx->tuning = std::move(t);
    return BEM_OK;
    BEM_CATCH
}

int bem_problem_tuning(const bem_problem* p, bem_tuning* out) {
    BEM_TRY
    if (!p || !out) fail(BEM_E_INVALID_ARG, "bad argument");
    *out = p->tune;
    return BEM_OK;
    BEM_CATCH
}

void bem_ctx_destroy(bem_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    {
        std::lock_guard<std::mutex> cap(capture_mutex());
        if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
        for (hipStream_t st : ctx->free_streams) (void)hipStreamDestroy(st);
        ctx->free_streams.clear();
        (void)hipDeviceSynchronize();
    }
    release_cached_device_memory(ctx->device);
    delete ctx;
    (void)hipGetLastError();   // nothing to report to: failures here leave no pending error
}

int bem_ctx_release_cached(bem_ctx* ctx) {
    BEM_TRY
    if (!ctx) fail(BEM_E_INVALID_ARG, "NULL ctx");
    set_device(ctx);
    release_cached_device_memory(ctx->device);
    HIP_CHECK(hipGetLastError());
    return BEM_OK;
    BEM_CATCH
}

int bem_ctx_synchronize(bem_ctx* ctx) {
    BEM_TRY
    if (!ctx) fail(BEM_E_INVALID_ARG, "NULL ctx");
    set_device(ctx);
    HIP_CHECK(hipDeviceSynchronize());
    return BEM_OK;
    BEM_CATCH
}

int bem_problem_bench_matvec(const bem_problem* p, int fp32, int32_t k, int reps, double* seconds) {
    BEM_TRY
    if (!p || !seconds || k <= 0 || reps <= 0) fail(BEM_E_INVALID_ARG, "bad argument");
    set_device(p->ctx);
    const int64_t N = p->N;
    if (N == 0) { *seconds = 0; return BEM_OK; }
    std::lock_guard<std::mutex> call(p->call_mu);
    DeviceBuffer x(sizeof(double) * N * k, p->stream), y(sizeof(double) * N * k, p->stream);
    std::vector<double> hx(size_t(N) * k);
    for (size_t i = 0; i < hx.size(); ++i) hx[i] = 1.0 / double(1 + (i % 97));
    HIP_CHECK(hipMemcpyAsync(x.ptr, hx.data(), sizeof(double) * hx.size(), hipMemcpyHostToDevice, p->stream));
    matvec_device(p, fp32 != 0, x.as<double>(), N, k, y.as<double>(), p->stream);   // warm-up
    hipEvent_t a, b;
    HIP_CHECK(hipEventCreate(&a));
    HIP_CHECK(hipEventCreate(&b));
    HIP_CHECK(hipEventRecord(a, p->stream));
    for (int r = 0; r < reps; ++r) matvec_device(p, fp32 != 0, x.as<double>(), N, k, y.as<double>(), p->stream);
    HIP_CHECK(hipEventRecord(b, p->stream));
    HIP_CHECK(hipEventSynchronize(b));
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *seconds = double(ms) * 1e-3 / reps;
    return BEM_OK;
    BEM_CATCH
}

int bem_mesh_analyze(const double* vertices, int64_t nv, const int32_t* triangles, int64_t nt, int64_t* n_dofs,
                     int32_t* dof_vertex, int32_t* dof_sector, int32_t* q) {
    BEM_TRY
    MeshTopo m;
    analyze_mesh(vertices, nv, triangles, nt, m);
    if (n_dofs) *n_dofs = m.N;
    if (dof_vertex && m.N) std::memcpy(dof_vertex, m.dof_vertex.data(), sizeof(int32_t) * m.N);
    if (dof_sector && m.N) std::memcpy(dof_sector, m.dof_sector.data(), sizeof(int32_t) * m.N);
    if (q) std::memcpy(q, m.q.data(), sizeof(int32_t) * nv);
    return BEM_OK;
    BEM_CATCH
}

int bem_assemble(bem_ctx* ctx, const double* vertices, int64_t nv, const int32_t* triangles, int64_t nt,
                 const bem_assemble_opts* opts, bem_problem** out) {
    return bem_assemble_dev(ctx, vertices, nullptr, nv, triangles, nullptr, nt, opts, out);
}

int bem_assemble_dev(bem_ctx* ctx, const double* vertices, const double* d_vertices, int64_t nv,
                     const int32_t* triangles, const int32_t* d_triangles, int64_t nt,
                     const bem_assemble_opts* opts, bem_problem** out) {
    BEM_TRY
    if (!ctx || !out) fail(BEM_E_INVALID_ARG, "ctx/out is NULL");
    *out = nullptr;
    set_device(ctx);
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<bem_problem> p(new bem_problem());
    p->ctx = ctx;
    p->tune = tuning_for(ctx->tuning, nt);
    p->near_order = (opts && opts->near_order > 0) ? opts->near_order : 10;
    if (p->near_order > 64) fail(BEM_E_INVALID_ARG, "near_order above 64");
    p->has_w32 = opts && opts->precision == BEM_FP32_REFINE;
    p->has_pairs = opts && opts->keep_pair_matrix;
    p->panel_rows = (opts && opts->pair_panel_rows > 0) ? opts->pair_panel_rows : 0;
    p->stream = acquire_stream(ctx);
    // locality order of a valid mesh (an invalid one is analysed as given, which reports its error)
    bool valid = vertices && triangles && nv > 0 && nt > 0 && nt <= (int64_t(1) << 30) && nv <= INT32_MAX;
    if (valid) {
        std::atomic<bool> bad{false};
        parallel_for(3 * nv, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i)
                if (!std::isfinite(vertices[i])) bad = true;
        }, 1 << 16);
        parallel_for(3 * nt, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i)
                if (triangles[i] < 0 || triangles[i] >= nv) bad = true;
        }, 1 << 16);
        valid = !bad;
    }
    std::vector<double> Vint;
    std::vector<int32_t> Tint, vert_int;
    DeviceBuffer dVint, dTint;
    if (valid && !(opts && opts->keep_order)) {
        locality_order(vertices, nv, triangles, nt, p->vert_user, p->tri_user);
        vert_int.resize(size_t(nv));
        p->tri_int.resize(size_t(nt));
        Vint.resize(size_t(3 * nv));
        Tint.resize(size_t(3 * nt));
        parallel_for(nv, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) {
                vert_int[size_t(p->vert_user[size_t(i)])] = int32_t(i);
                for (int c = 0; c < 3; ++c) Vint[size_t(3 * i + c)] = vertices[3 * int64_t(p->vert_user[size_t(i)]) + c];
            }
        }, 8192);
        parallel_for(nt, [&](int64_t lo, int64_t hi) {
            for (int64_t t = lo; t < hi; ++t) {
                p->tri_int[size_t(p->tri_user[size_t(t)])] = int32_t(t);
                for (int a = 0; a < 3; ++a)
                    Tint[size_t(3 * t + a)] = vert_int[size_t(triangles[3 * int64_t(p->tri_user[size_t(t)]) + a])];
            }
        }, 8192);
        p->renumbered = true;
    }
    const double* Vp = p->renumbered ? Vint.data() : vertices;
    const int32_t* Tp = p->renumbered ? Tint.data() : triangles;
    const double* dVp = d_vertices;
    const int32_t* dTp = d_triangles;
    try {
        if (p->renumbered && d_vertices && d_triangles) {
            // renumbered device copies from the caller's, on the device (only the index maps go up)
            DeviceBuffer dvu = upload(p->vert_user, p->stream), dvi = upload(vert_int, p->stream), dtu = upload(p->tri_user, p->stream);
            dVint = DeviceBuffer(sizeof(double) * 3 * nv, p->stream);
            dTint = DeviceBuffer(sizeof(int32_t) * 3 * nt, p->stream);
            renumber_mesh_device(d_vertices, d_triangles, nv, nt, dvu.as<int32_t>(), dvi.as<int32_t>(), dtu.as<int32_t>(),
                                 dVint.as<double>(), dTint.as<int32_t>(), p->stream);
            dVp = dVint.as<double>();
            dTp = dTint.as<int32_t>();
        } else if (p->renumbered) {
            dVp = nullptr;
            dTp = nullptr;
        }
        assemble_device(p.get(), Vp, nv, Tp, nt, [&](NearList& near) {
            analyze_mesh(Vp, nv, Tp, nt, p->topo, p->renumbered ? p->tri_user.data() : nullptr,
                         p->renumbered ? p->vert_user.data() : nullptr);
            build_near_list(p->topo, near, p->renumbered ? p->tri_user.data() : nullptr);
            p->N = p->topo.N;
        }, dVp, dTp);
        if (p->renumbered) {
            // internal dof (vertex i, label j) is the caller's dof (vert_user[i], j): the labels agree
            // because the stars listed their triangles in the caller's order
            const MeshTopo& m = p->topo;
            std::vector<int64_t> first_user(size_t(nv) + 1, 0);
            for (int64_t u = 0; u < nv; ++u) first_user[size_t(u) + 1] = first_user[size_t(u)] + std::max(0, m.q[size_t(vert_int[size_t(u)])] - 1);
            p->dof_user.resize(size_t(p->N));
            p->dof_int.resize(size_t(p->N));
            for (int64_t d = 0; d < p->N; ++d) {
                const int64_t du = first_user[size_t(p->vert_user[size_t(m.dof_vertex[size_t(d)])])] + m.dof_sector[size_t(d)];
                p->dof_user[size_t(d)] = int32_t(du);
                p->dof_int[size_t(du)] = int32_t(d);
            }
            p->d_dof_user = upload(p->dof_user, p->stream);   // from the problem's own copies, which outlive the copy
            p->d_dof_int = upload(p->dof_int, p->stream);
        }
    } catch (...) {
        // device work already queued must end before its buffers go
        (void)hipStreamSynchronize(p->stream);
        hipStream_t s = p->stream, s2 = p->aux_stream;
        if (s2) (void)hipStreamSynchronize(s2);
        p.reset();
        release_stream(ctx, s);
        release_stream(ctx, s2);
        throw;
    }
    p->bytes = int64_t(p->W64.bytes + p->W32.bytes + p->I.bytes + p->normal.bytes + p->area.bytes + p->dof_ptr.bytes +
                       p->dof_tri.bytes + p->dof_c.bytes + p->tri_ptr.bytes + p->tri_dof.bytes + p->tri_corner.bytes +
                       p->tri_c.bytes + p->mv_xt.bytes + p->mv_partial.bytes + p->mv_tiles[0].bytes + p->mv_tiles[1].bytes + p->mv_sym.bytes);
    p->t_assemble = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = p.release();
    return BEM_OK;
    BEM_CATCH
}

int bem_mesh_analyze_2d(const double* vertices, int64_t nv, const int32_t* segments, int64_t ns, int64_t* n_dofs,
                        int32_t* dof_vertex, int32_t* dof_sector, int32_t* q, double* c) {
    BEM_TRY
    MeshTopo m;
    analyze_segments(vertices, nv, segments, ns, m);
    if (n_dofs) *n_dofs = m.N;
    if (dof_vertex && m.N) std::memcpy(dof_vertex, m.dof_vertex.data(), sizeof(int32_t) * m.N);
    if (dof_sector && m.N) std::memcpy(dof_sector, m.dof_sector.data(), sizeof(int32_t) * m.N);
    if (q) std::memcpy(q, m.q.data(), sizeof(int32_t) * nv);
    if (c) {
        std::memset(c, 0, sizeof(double) * ns * 2 * m.N);
        for (int64_t t = 0; t < ns; ++t)
            for (int64_t e = m.tri_ptr[t]; e < m.tri_ptr[t + 1]; ++e)
                c[(t * 2 + m.tri_corner[e]) * m.N + m.tri_dof[e]] = double(m.tri_c[e]);
    }
    return BEM_OK;
    BEM_CATCH
}

int bem_assemble_2d(bem_ctx* ctx, const double* vertices, int64_t nv, const int32_t* segments, int64_t ns,
                    const bem_assemble_opts* opts, bem_problem** out) {
    BEM_TRY
    if (!ctx || !out) fail(BEM_E_INVALID_ARG, "ctx/out is NULL");
    *out = nullptr;
    set_device(ctx);
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<bem_problem> p(new bem_problem());
    p->ctx = ctx;
    p->tune = tuning_for(ctx->tuning, ns);
    p->has_w32 = opts && opts->precision == BEM_FP32_REFINE;
    if (opts && opts->keep_pair_matrix) fail(BEM_E_INVALID_ARG, "keep_pair_matrix is for triangle meshes");
    p->stream = acquire_stream(ctx);
    try {
        assemble_2d_device(p.get(), vertices, nv, segments, ns);
    } catch (...) {
        (void)hipStreamSynchronize(p->stream);
        hipStream_t s = p->stream, s2 = p->aux_stream;
        if (s2) (void)hipStreamSynchronize(s2);
        p.reset();
        release_stream(ctx, s);
        release_stream(ctx, s2);
        throw;
    }
    p->bytes = int64_t(p->W64.bytes + p->W32.bytes + p->normal.bytes + p->area.bytes + p->dof_ptr.bytes +
                       p->dof_tri.bytes + p->dof_c.bytes + p->tri_ptr.bytes + p->tri_dof.bytes + p->tri_corner.bytes +
                       p->tri_c.bytes + p->mv_xt.bytes + p->mv_partial.bytes + p->mv_tiles[0].bytes + p->mv_tiles[1].bytes + p->mv_sym.bytes);
    p->t_assemble = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = p.release();
    return BEM_OK;
    BEM_CATCH
}

void bem_problem_destroy(bem_problem* p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->aux_stream) (void)hipStreamSynchronize(p->aux_stream);
    for (hipEvent_t& e : p->ev_contract)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->ev_spans)
        if (e) (void)hipEventDestroy(e);
    hipStream_t s = p->stream, s2 = p->aux_stream;
    bem_ctx* ctx = p->ctx;
    delete p;
    release_stream(ctx, s2);
    release_stream(ctx, s);
    (void)hipGetLastError();
}

int bem_problem_get_info(const bem_problem* p, bem_problem_info* info) {
    BEM_TRY
    if (!p || !info) fail(BEM_E_INVALID_ARG, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->n_dofs = p->N;
    info->n_tri = p->topo.nt;
    info->n_vert = p->topo.nv;
    info->n_near_pairs = p->n_near;
    info->bytes_device = p->bytes;
    for (int32_t q : p->topo.q) info->q_hist[std::min(q, 15)] += 1;
    info->t_assemble_s = p->t_assemble;
    std::lock_guard<std::mutex> lk(p->info_mu);
    if (!p->ev_spans.empty()) {   // the panels' phase times, once the last contraction has finished
        set_device(p->ctx);
        const hipError_t q = hipEventQuery(p->ev_spans.back());
        if (q == hipSuccess) {
            double t[3] = {0.0, 0.0, 0.0};
            for (size_t i = 0; i + 1 < p->ev_spans.size(); i += 2) {
                float ms = 0.f;
                HIP_CHECK(hipEventElapsedTime(&ms, p->ev_spans[i], p->ev_spans[i + 1]));
                t[(i / 2) % 3] += ms * 1e-3;
            }
            p->t_far = t[0];
            p->t_near = t[1];
            p->t_contract = t[2];
            for (hipEvent_t e : p->ev_spans) (void)hipEventDestroy(e);
            p->ev_spans.clear();
        } else if (q == hipErrorNotReady) {
            (void)hipGetLastError();
        } else {
            HIP_CHECK(q);
        }
    }
    const bool pending = !p->ev_spans.empty();
    info->t_far_s = pending ? std::nan("") : p->t_far;
    info->t_near_s = pending ? std::nan("") : p->t_near;
    if (p->ev_contract[1]) {   // the contraction's time, once it has finished (the call never waits)
        set_device(p->ctx);
        const hipError_t q = hipEventQuery(p->ev_contract[1]);
        if (q == hipSuccess) {
            float ms = 0.f;
            HIP_CHECK(hipEventElapsedTime(&ms, p->ev_contract[0], p->ev_contract[1]));
            p->t_contract = ms * 1e-3;
            (void)hipEventDestroy(p->ev_contract[0]);
            (void)hipEventDestroy(p->ev_contract[1]);
            p->ev_contract[0] = p->ev_contract[1] = nullptr;
        } else if (q == hipErrorNotReady) {
            (void)hipGetLastError();
        } else {
            HIP_CHECK(q);
        }
    }
    info->t_contract_s = (p->ev_contract[1] || pending) ? std::nan("") : p->t_contract;
    info->t_host_s = p->t_host;
    info->n_pair_panels = p->n_panels;
    info->dim = p->topo.dim;
    info->panels_replanned = p->panels_replanned;
    return BEM_OK;
    BEM_CATCH
}

int bem_problem_dofs(const bem_problem* p, int32_t* dof_vertex, int32_t* dof_sector) {
    BEM_TRY
    if (!p) fail(BEM_E_INVALID_ARG, "NULL problem");
    for (int64_t u = 0; u < p->N; ++u) {
        const int64_t d = p->renumbered ? p->dof_int[size_t(u)] : u;
        const int32_t v = p->topo.dof_vertex[size_t(d)];
        if (dof_vertex) dof_vertex[u] = p->renumbered ? p->vert_user[size_t(v)] : v;
        if (dof_sector) dof_sector[u] = p->topo.dof_sector[size_t(d)];
    }
    return BEM_OK;
    BEM_CATCH
}

int bem_problem_copy_matrix(const bem_problem* p, int64_t row0, int64_t nrows, double* out) {
    BEM_TRY
    if (!p || !out) fail(BEM_E_INVALID_ARG, "NULL argument");
    if (row0 < 0 || nrows < 0 || row0 + nrows > p->N) fail(BEM_E_INVALID_ARG, "row range outside the matrix");
    set_device(p->ctx);
    if (nrows == 0) return BEM_OK;
    if (p->renumbered) {
        std::vector<int64_t> rows(static_cast<size_t>(nrows));
        for (int64_t i = 0; i < nrows; ++i) rows[size_t(i)] = row0 + i;
        copy_rows_user(p, rows.data(), nrows, out);
        return BEM_OK;
    }
    // stream-ordered behind the contraction that may still be writing W (no null-stream copy: it
    // could wait on work of other threads' streams)
    HIP_CHECK(hipMemcpy2DAsync(out, sizeof(double) * p->N, p->W64.as<double>() + row0 * p->ldw, sizeof(double) * p->ldw,
                               sizeof(double) * p->N, size_t(nrows), hipMemcpyDeviceToHost, p->stream));
    HIP_CHECK(hipStreamSynchronize(p->stream));
    return BEM_OK;
    BEM_CATCH
}

int bem_problem_copy_rows(const bem_problem* p, const int64_t* rows, int64_t nrows, double* out) {
    BEM_TRY
    if (!p || (!rows && nrows) || (!out && nrows)) fail(BEM_E_INVALID_ARG, "NULL argument");
    set_device(p->ctx);
    for (int64_t i = 0; i < nrows; ++i)
        if (rows[i] < 0 || rows[i] >= p->N) fail(BEM_E_INVALID_ARG, "row index out of range");
    if (p->renumbered) {
        copy_rows_user(p, rows, nrows, out);
        return BEM_OK;
    }
    // stream-ordered behind the contraction that may still be writing W
    for (int64_t i = 0; i < nrows; ++i)
        HIP_CHECK(hipMemcpyAsync(out + i * p->N, p->W64.as<double>() + rows[i] * p->ldw, sizeof(double) * p->N,
                                 hipMemcpyDeviceToHost, p->stream));
    HIP_CHECK(hipStreamSynchronize(p->stream));
    return BEM_OK;
    BEM_CATCH
}

int bem_problem_pair_integrals(const bem_problem* p, const int32_t* pairs, int64_t npairs, double* out) {
    BEM_TRY
    if (!p || (!pairs && npairs) || (!out && npairs)) fail(BEM_E_INVALID_ARG, "NULL argument");
    if (!p->has_pairs || !p->I.ptr) fail(BEM_E_INVALID_ARG, "assemble with keep_pair_matrix = 1");
    set_device(p->ctx);
    const int64_t nt = p->topo.nt;
    for (int64_t i = 0; i < npairs; ++i) {
        const int64_t a = pairs[2 * i], b = pairs[2 * i + 1];
        if (a < 0 || a >= nt || b < 0 || b >= nt) fail(BEM_E_INVALID_ARG, "pair index out of range");
    }
    auto tri = [&](int64_t t) { return p->renumbered ? int64_t(p->tri_int[size_t(t)]) : t; };
    for (int64_t i = 0; i < npairs; ++i)
        HIP_CHECK(hipMemcpyAsync(out + i, p->I.as<double>() + tri(pairs[2 * i]) * p->ldI + tri(pairs[2 * i + 1]), sizeof(double),
                                 hipMemcpyDeviceToHost, p->stream));
    HIP_CHECK(hipStreamSynchronize(p->stream));
    return BEM_OK;
    BEM_CATCH
}

int bem_rhs(const bem_problem* p, const double* g, int32_t k, double* out) {
    BEM_TRY
    if (!p || !g || !out || k <= 0) fail(BEM_E_INVALID_ARG, "bad argument");
    set_device(p->ctx);
    const int64_t N = p->N;
    if (N == 0) return BEM_OK;
    DeviceBuffer dg(sizeof(double) * 3 * k, p->stream), dL(sizeof(double) * N * k, p->stream);
    HIP_CHECK(hipMemcpyAsync(dg.ptr, g, sizeof(double) * 3 * k, hipMemcpyHostToDevice, p->stream));
    rhs_device(p, dg.as<double>(), k, dL.as<double>(), p->stream);
    DeviceBuffer dLu(sizeof(double) * N * k, p->stream);
    dofs_to_user(p, dL.as<double>(), dLu.as<double>(), k);
    HIP_CHECK(hipMemcpyAsync(out, dLu.ptr, sizeof(double) * N * k, hipMemcpyDeviceToHost, p->stream));
    HIP_CHECK(hipStreamSynchronize(p->stream));
    return BEM_OK;
    BEM_CATCH
}

int bem_matvec(const bem_problem* p, const double* x, int32_t k, int fp32, double* y) {
    BEM_TRY
    if (!p || !x || !y || k <= 0) fail(BEM_E_INVALID_ARG, "bad argument");
    set_device(p->ctx);
    const int64_t N = p->N;
    if (N == 0) return BEM_OK;
    std::lock_guard<std::mutex> call(p->call_mu);
    DeviceBuffer dx(sizeof(double) * N * k, p->stream), dy(sizeof(double) * N * k, p->stream);
    DeviceBuffer du(sizeof(double) * N * k, p->stream);   // the caller's order
    HIP_CHECK(hipMemcpyAsync(du.ptr, x, sizeof(double) * N * k, hipMemcpyHostToDevice, p->stream));
    dofs_to_internal(p, du.as<double>(), dx.as<double>(), k);
    matvec_device(p, fp32 != 0, dx.as<double>(), N, k, dy.as<double>(), p->stream);
    dofs_to_user(p, dy.as<double>(), du.as<double>(), k);
    HIP_CHECK(hipMemcpyAsync(y, du.ptr, sizeof(double) * N * k, hipMemcpyDeviceToHost, p->stream));
    HIP_CHECK(hipStreamSynchronize(p->stream));
    return BEM_OK;
    BEM_CATCH
}

int bem_matvec_noalloc(const bem_problem* p, const double* d_x, int32_t k, int fp32, double* d_y) {
    BEM_TRY
    if (!p || !d_x || !d_y || k <= 0) fail(BEM_E_INVALID_ARG, "bad argument");
    set_device(p->ctx);
    const int64_t N = p->N;
    if (N == 0) return BEM_OK;
    if (fp32 && !p->W32.ptr) fail(BEM_E_INVALID_ARG, "problem has no FP32 matrix (assemble with BEM_FP32_REFINE)");
    const size_t need = noalloc_matvec_bytes(p, fp32 != 0, k);
    if (need > kNoAllocScratchBytes)
        fail(BEM_E_INVALID_ARG, "bem_matvec_noalloc: this product needs " + std::to_string(need) +
                                    " bytes of scratch, more than the " + std::to_string(kNoAllocScratchBytes) +
                                    " it has (use bem_matvec)");
    void* scr = noalloc_scratch_address(p->ctx->device);
    std::lock_guard<std::mutex> call(p->call_mu);
    matvec_device_noalloc(p, fp32 != 0, d_x, N, k, d_y, p->stream, scr);
    HIP_CHECK(hipStreamSynchronize(p->stream));
    return BEM_OK;
    BEM_CATCH
}

int bem_jump_values(const bem_problem* p, const double* phi, double* jump_out) {
    BEM_TRY
    if (!p || !phi || !jump_out) fail(BEM_E_INVALID_ARG, "bad argument");
    set_device(p->ctx);
    const int64_t N = p->N, nt = p->topo.nt, corners = p->topo.dim == 2 ? 2 : 3;
    DeviceBuffer dp(sizeof(double) * std::max<int64_t>(1, N), p->stream), dj(sizeof(double) * nt * corners, p->stream);
    DeviceBuffer du(sizeof(double) * std::max<int64_t>(1, N), p->stream);
    if (N) {
        HIP_CHECK(hipMemcpyAsync(du.ptr, phi, sizeof(double) * N, hipMemcpyHostToDevice, p->stream));
        dofs_to_internal(p, du.as<double>(), dp.as<double>(), 1);
    }
    jump_values_device(p, dp.as<double>(), dj.as<double>(), p->stream);
    std::vector<double> tmp(p->renumbered ? size_t(nt * corners) : 0);
    HIP_CHECK(hipMemcpyAsync(p->renumbered ? tmp.data() : jump_out, dj.ptr, sizeof(double) * nt * corners, hipMemcpyDeviceToHost,
                             p->stream));
    HIP_CHECK(hipStreamSynchronize(p->stream));
    if (p->renumbered)   // per triangle of the caller's numbering (corners in the caller's order too)
        for (int64_t t = 0; t < nt; ++t)
            for (int64_t a = 0; a < corners; ++a) jump_out[t * corners + a] = tmp[size_t(p->tri_int[size_t(t)] * corners + a)];
    return BEM_OK;
    BEM_CATCH
}

int bem_double_layer(bem_problem* p, const double* phi, int32_t k, const double* targets, int64_t m, double* u_out) {
    BEM_TRY
    if (!p || !phi || !targets || !u_out || k < 1 || m < 0) fail(BEM_E_INVALID_ARG, "bad argument");
    for (int64_t i = 0; i < 3 * m; ++i)
        if (!std::isfinite(targets[i])) fail(BEM_E_INVALID_ARG, "non-finite target coordinate");
    set_device(p->ctx);
    if (m == 0) return BEM_OK;
    const int64_t N = p->N;
    std::lock_guard<std::mutex> call(p->call_mu);
    DeviceBuffer dp(sizeof(double) * std::max<int64_t>(1, N * k), p->stream), dx(sizeof(double) * 3 * m, p->stream),
        du(sizeof(double) * k * m, p->stream);
    DeviceBuffer dpu(sizeof(double) * std::max<int64_t>(1, N * k), p->stream);   // phi in the caller's order
    if (N) {
        HIP_CHECK(hipMemcpyAsync(dpu.ptr, phi, sizeof(double) * N * k, hipMemcpyHostToDevice, p->stream));
        dofs_to_internal(p, dpu.as<double>(), dp.as<double>(), k);
    }
    HIP_CHECK(hipMemcpyAsync(dx.ptr, targets, sizeof(double) * 3 * m, hipMemcpyHostToDevice, p->stream));
    double_layer_device(p, dp.as<double>(), k, dx.as<double>(), m, du.as<double>(), p->stream);
    HIP_CHECK(hipMemcpyAsync(u_out, du.ptr, sizeof(double) * k * m, hipMemcpyDeviceToHost, p->stream));
    HIP_CHECK(hipStreamSynchronize(p->stream));
    return BEM_OK;
    BEM_CATCH
}

int bem_precond_setup(bem_problem* p, const int32_t* patch_of_triangle, const double* coarse_vertices, int64_t ncv,
                      const int32_t* coarse_triangles, int64_t nct, const int32_t* coarse_of_triangle,
                      const bem_precond_opts* opts, bem_precond** out) {
    BEM_TRY
    if (!p || !out) fail(BEM_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (p->topo.dim != 3) fail(BEM_E_INVALID_ARG, "bem_precond_setup needs a triangle mesh; use bem_precond_setup_2d");
    set_device(p->ctx);
    std::unique_ptr<bem_precond> m(new bem_precond());
    m->p = p;
    m->use_coarse = opts ? opts->use_coarse != 0 : true;
    m->fp32 = opts ? opts->factor_fp32 != 0 : false;
    if (opts && (opts->wirebasket < 0 || opts->wirebasket > 1)) fail(BEM_E_INVALID_ARG, "wirebasket must be 0 or 1");
    m->wb_diag = opts ? opts->wirebasket == 1 : false;
    m->diag_shift = opts ? opts->diag_shift : 0.0;
    if (!std::isfinite(m->diag_shift)) fail(BEM_E_INVALID_ARG, "diag_shift is not finite");
    // per-triangle inputs in the problem's triangle order
    std::vector<int32_t> patch_int, coarse_int;
    if (p->renumbered) {
        const int64_t nt = p->topo.nt;
        if (patch_of_triangle) {
            patch_int.resize(size_t(nt));
            for (int64_t t = 0; t < nt; ++t) patch_int[size_t(t)] = patch_of_triangle[p->tri_user[size_t(t)]];
            patch_of_triangle = patch_int.data();
        }
        if (coarse_of_triangle) {
            coarse_int.resize(size_t(nt));
            for (int64_t t = 0; t < nt; ++t) coarse_int[size_t(t)] = coarse_of_triangle[p->tri_user[size_t(t)]];
            coarse_of_triangle = coarse_int.data();
        }
    }
    std::lock_guard<std::mutex> call(p->call_mu);
    precond_setup_device(m.get(), patch_of_triangle, coarse_vertices, ncv, coarse_triangles, nct, coarse_of_triangle);
    *out = m.release();
    return BEM_OK;
    BEM_CATCH
}

int bem_precond_setup_2d(bem_problem* p, const int32_t* patch_of_segment, const double* coarse_vertices, int64_t ncv,
                         const int32_t* coarse_segments, int64_t ncs, const int32_t* coarse_of_segment,
                         const bem_precond_opts* opts, bem_precond** out) {
    BEM_TRY
    if (!p || !out) fail(BEM_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (p->topo.dim != 2) fail(BEM_E_INVALID_ARG, "bem_precond_setup_2d needs a segment mesh");
    set_device(p->ctx);
    std::unique_ptr<bem_precond> m(new bem_precond());
    m->p = p;
    m->use_coarse = opts ? opts->use_coarse != 0 : true;
    m->fp32 = opts ? opts->factor_fp32 != 0 : false;
    if (opts && (opts->wirebasket < 0 || opts->wirebasket > 1)) fail(BEM_E_INVALID_ARG, "wirebasket must be 0 or 1");
    m->wb_diag = opts ? opts->wirebasket == 1 : false;
    m->diag_shift = opts ? opts->diag_shift : 0.0;
    if (!std::isfinite(m->diag_shift)) fail(BEM_E_INVALID_ARG, "diag_shift is not finite");
    std::lock_guard<std::mutex> call(p->call_mu);
    precond_setup_device(m.get(), patch_of_segment, coarse_vertices, ncv, coarse_segments, ncs, coarse_of_segment);
    *out = m.release();
    return BEM_OK;
    BEM_CATCH
}

void bem_precond_destroy(bem_precond* m) {
    if (!m) return;
    (void)hipSetDevice(m->p->ctx->device);
    (void)hipStreamSynchronize(m->p->stream);
    delete m;
    (void)hipGetLastError();
}

int bem_precond_sizes(const bem_precond* m, int64_t* n_faces, int64_t* n_wb, int64_t* n_coarse, int64_t* max_face) {
    BEM_TRY
    if (!m) fail(BEM_E_INVALID_ARG, "NULL preconditioner");
    if (n_faces) *n_faces = m->n_faces;
    if (n_wb) *n_wb = m->n_wb;
    if (n_coarse) *n_coarse = m->nH;
    if (max_face) *max_face = m->max_face;
    return BEM_OK;
    BEM_CATCH
}

int bem_precond_apply(const bem_precond* m, const double* r, int32_t k, double* z) {
    BEM_TRY
    if (!m || !r || !z || k <= 0) fail(BEM_E_INVALID_ARG, "bad argument");
    const bem_problem* p = m->p;
    set_device(p->ctx);
    const int64_t N = p->N;
    std::lock_guard<std::mutex> call(p->call_mu);
    DeviceBuffer dr(sizeof(double) * N * k, m->p->stream), dz(sizeof(double) * N * k, m->p->stream);
    DeviceBuffer scr(sizeof(double) * precond_scratch_size(m, std::min(k, 16)), m->p->stream);
    DeviceBuffer du(sizeof(double) * N * k, m->p->stream);
    HIP_CHECK(hipMemcpyAsync(du.ptr, r, sizeof(double) * N * k, hipMemcpyHostToDevice, p->stream));
    dofs_to_internal(p, du.as<double>(), dr.as<double>(), k);
    precond_apply_device(m, false, dr.as<double>(), N, k, dz.as<double>(), p->stream, scr.as<double>());
    dofs_to_user(p, dz.as<double>(), du.as<double>(), k);
    HIP_CHECK(hipMemcpyAsync(z, du.ptr, sizeof(double) * N * k, hipMemcpyDeviceToHost, p->stream));
    HIP_CHECK(hipStreamSynchronize(p->stream));
    return BEM_OK;
    BEM_CATCH
}

int bem_pcg_solve(bem_problem* p, const bem_precond* m, const double* g, int32_t k, const bem_solve_opts* opts,
                  double* phi_out, bem_solve_info* info) {
    BEM_TRY
    if (!p || !g || k <= 0) fail(BEM_E_INVALID_ARG, "bad argument");
    set_device(p->ctx);
    const int64_t N = p->N;
    DeviceBuffer dg(sizeof(double) * 3 * k, p->stream), dL(sizeof(double) * std::max<int64_t>(1, N * k), p->stream);
    HIP_CHECK(hipMemcpyAsync(dg.ptr, g, sizeof(double) * 3 * k, hipMemcpyHostToDevice, p->stream));
    rhs_device(p, dg.as<double>(), k, dL.as<double>(), p->stream);
    return solve_common(p, m, dL.as<double>(), k, opts, phi_out, info);
    BEM_CATCH
}

int bem_pcg_solve_dev(bem_problem* p, const bem_precond* m, const double* g, int32_t k, const bem_solve_opts* opts,
                      double* d_phi_out, bem_solve_info* info) {
    BEM_TRY
    if (!p || !g || k <= 0 || !d_phi_out) fail(BEM_E_INVALID_ARG, "bad argument");
    set_device(p->ctx);
    const int64_t N = p->N;
    DeviceBuffer dg(sizeof(double) * 3 * k, p->stream), dL(sizeof(double) * std::max<int64_t>(1, N * k), p->stream);
    HIP_CHECK(hipMemcpyAsync(dg.ptr, g, sizeof(double) * 3 * k, hipMemcpyHostToDevice, p->stream));
    rhs_device(p, dg.as<double>(), k, dL.as<double>(), p->stream);
    return solve_common(p, m, dL.as<double>(), k, opts, nullptr, info, d_phi_out);
    BEM_CATCH
}

int bem_pcg_solve_rhs(bem_problem* p, const bem_precond* m, const double* rhs, int32_t k, const bem_solve_opts* opts,
                      double* phi_out, bem_solve_info* info) {
    BEM_TRY
    if (!p || !rhs || k <= 0) fail(BEM_E_INVALID_ARG, "bad argument");
    set_device(p->ctx);
    const int64_t N = p->N;
    DeviceBuffer dL(sizeof(double) * std::max<int64_t>(1, N * k), p->stream), du(sizeof(double) * std::max<int64_t>(1, N * k), p->stream);
    if (N) {
        HIP_CHECK(hipMemcpyAsync(du.ptr, rhs, sizeof(double) * N * k, hipMemcpyHostToDevice, p->stream));
        dofs_to_internal(p, du.as<double>(), dL.as<double>(), k);
    }
    return solve_common(p, m, dL.as<double>(), k, opts, phi_out, info);
    BEM_CATCH
}

}  // extern "C"
