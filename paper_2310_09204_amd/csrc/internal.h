// Internal declarations of libbem (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bem.h"

namespace bem {

// the tuning entry for a mesh of nt triangles, defaults filled in
bem_tuning tuning_for(const std::vector<bem_tuning>& table, int64_t nt);

struct Failure {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);
void set_last_error(const std::string& msg);

#define HIP_CHECK(expr)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            ::bem::fail(BEM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------------------------------
// Host topology of a multiscreen mesh (Section 4.2 / 4.3 of the paper)
// ------------------------------------------------------------------------------------------
struct MeshTopo {
    int dim = 3;                    // 3: triangles in space; 2: segments in the plane (nt counts segments)
    int64_t nv = 0, nt = 0, N = 0;
    std::vector<double> V;          // nv*3 (z = 0 in the plane)
    std::vector<int32_t> T;         // nt*3 (triangles)
    std::vector<int32_t> S;         // nt*2 (segments)
    std::vector<double> normal;     // nt*3 unit normal n_T
    std::vector<double> area;       // nt
    std::vector<int32_t> q;         // nv sector counts
    std::vector<int32_t> sector;    // nt*2*3: label of side s of triangle t at its corner a
    std::vector<int64_t> first_dof; // nv+1: dofs of vertex v are first_dof[v] .. first_dof[v+1]-1
    std::vector<int32_t> dof_vertex, dof_sector;
    // triangle -> (dof, corner, c) with c = s_+ - s_- (jump coefficient), CSR over triangles
    std::vector<int64_t> tri_ptr;
    std::vector<int32_t> tri_dof;
    std::vector<int8_t> tri_corner, tri_c;
    // dof -> (triangle, corner, c), CSR over dofs
    std::vector<int64_t> dof_ptr;
    std::vector<int32_t> dof_tri;
    std::vector<int8_t> dof_corner, dof_c;
};

// Validates and analyses a mesh; throws Failure with a BEM_E_* code on invalid input.
// tri_user / vert_user (optional): the caller's index of each triangle / vertex of a renumbered
// mesh.  Stars then list their triangles in the caller's order, so that sectors get the labels (and
// the reference sector) that the caller's numbering gives them, and errors name the caller's indices.
void analyze_mesh(const double* V, int64_t nv, const int32_t* T, int64_t nt, MeshTopo& out,
                  const int32_t* tri_user = nullptr, const int32_t* vert_user = nullptr);
// The same for a segment mesh in the plane (V: nv*2, S: ns*2): sectors are the angular regions
// between the segments at a vertex; normal (nt*3) holds n_s = (-tau_y, tau_x, 0), area the lengths,
// and the element CSR (tri_*) has corners 0 and 1.
void analyze_segments(const double* V, int64_t nv, const int32_t* S, int64_t ns, MeshTopo& out);

// Pairs of triangles with at least one common vertex, t1 <= t2, with the canonical vertex order
// the Duffy rules expect: type 3 (same triangle) A,B,C; type 2 (common edge A-B) A,B,C,C';
// type 1 (common vertex A) A,B,C,B',C'.
struct NearList {
    std::vector<int32_t> t1, t2;
    std::vector<int8_t> type;
    std::vector<int32_t> verts;     // 5 per pair (-1 where unused)
    int64_t count[4] = {0, 0, 0, 0};
};
// tri_user (optional): the caller's triangle indices of a renumbered mesh; each pair is then listed
// with its first triangle the one of smaller caller index (the near rules are not symmetric)
void build_near_list(const MeshTopo& m, NearList& out, const int32_t* tri_user = nullptr);

// Quadrature tables computed from their definitions
void triangle7_rule(double bary[7][3], double w[7]);
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);

// ------------------------------------------------------------------------------------------
// Device-side objects behind the opaque C handles
// ------------------------------------------------------------------------------------------
// Device allocation through a per-device cache: a released buffer is kept for reuse instead of
// being given back with hipFree, which synchronises the whole device (and can stall for hundreds
// of milliseconds on tens of GB).  Buffers below kPooledBytes are rounded up to a power of two and
// reused by exact size class; larger ones are reused if at most 25 % larger than the request.
// A buffer allocated for a stream is released stream-ordered: an event is recorded on that
// stream and the memory is handed out again only once the event has completed, so queued kernels
// that still read it are safe even when another thread allocates meanwhile.  A buffer with no
// stream must only be released when no queued work uses it.  Cached memory is given back when an
// allocation runs out of memory and when a context of the device is destroyed.
//
// Device-wide synchronising calls (hipFree, hipStreamDestroy) invalidate a HIP graph capture in
// progress on any stream, so they and the capture of a PCG iteration hold capture_mutex().
std::mutex& capture_mutex();

// Puts the calling thread in relaxed stream-capture interaction mode for its lifetime (restoring
// the previous mode after).  Library calls run concurrently on several host threads (the serving
// loop's workers, or callers' own threads) while one of them captures a PCG iteration into a HIP
// graph; in the default global mode the runtime may refuse allocations and synchronous copies on
// the other threads during such a capture.
struct RelaxedCapture {
    hipStreamCaptureMode prev = hipStreamCaptureModeRelaxed;
    RelaxedCapture() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
    ~RelaxedCapture() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
    RelaxedCapture(const RelaxedCapture&) = delete;
    RelaxedCapture& operator=(const RelaxedCapture&) = delete;
};

constexpr size_t kPooledBytes = size_t(64) << 20;
void release_cached_device_memory(int device);
// free device memory as the runtime reports it plus what the pool holds for reuse (which a
// large allocation gets back by releasing the cache when the runtime runs out)
size_t available_device_bytes(int device);

struct DeviceBuffer {
    void* ptr = nullptr;
    size_t bytes = 0;     // requested size
    size_t cap = 0;       // allocated size (>= bytes for a buffer reused from the cache)
    int dev = 0;
    bool pooled = false;
    hipStream_t stream = nullptr;   // stream whose queued work may use the buffer (release is ordered after it)
    DeviceBuffer() = default;
    DeviceBuffer(size_t b, hipStream_t s);
    ~DeviceBuffer();
    DeviceBuffer(const DeviceBuffer&) = delete;
    DeviceBuffer& operator=(const DeviceBuffer&) = delete;
    DeviceBuffer(DeviceBuffer&& o) noexcept
        : ptr(o.ptr), bytes(o.bytes), cap(o.cap), dev(o.dev), pooled(o.pooled), stream(o.stream) {
        o.ptr = nullptr;
        o.bytes = o.cap = 0;
        o.pooled = false;
        o.stream = nullptr;
    }
    DeviceBuffer& operator=(DeviceBuffer&& o) noexcept;
    void reset();
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

template <class T>
DeviceBuffer upload(const std::vector<T>& v, hipStream_t s) {
    DeviceBuffer b(std::max<size_t>(1, v.size()) * sizeof(T), s);
    if (!v.empty()) HIP_CHECK(hipMemcpyAsync(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return b;
}

// First failure of a parallel pass, kept by smallest position so the reported error does not depend
// on thread timing.
struct FirstFailure {
    std::mutex mu;
    int64_t pos = -1;
    Failure f{0, ""};
    void record(int64_t where, const Failure& x) {
        std::lock_guard<std::mutex> lk(mu);
        if (pos < 0 || where < pos) { pos = where; f = x; }
    }
    void rethrow() const { if (pos >= 0) throw f; }
};

// Runs fn(begin, end) over [0, n) split across a few host threads (at most 16); every range but
// the last starts at a multiple of grain.  fn must not throw.
template <class Fn>
void parallel_for(int64_t n, Fn&& fn, int64_t grain = 2048) {
    const int64_t hw = std::max<int64_t>(1, std::min<int64_t>(16, std::thread::hardware_concurrency()));
    const int64_t nth = std::max<int64_t>(1, std::min<int64_t>(hw, n / grain));
    if (nth == 1) {
        fn(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = ((n + nth - 1) / nth + grain - 1) / grain * grain;
    for (int64_t k = 0; k < nth; ++k) {
        const int64_t b = k * chunk, e = std::min(n, b + chunk);
        if (b < e) th.emplace_back([&fn, b, e] { fn(b, e); });
    }
    for (auto& t : th) t.join();
}

// Sorts [first, first + n) under a strict total order on a few host threads: chunks sorted in
// parallel, then merged pairwise (a strict total order has one sorted order, whatever the split).
template <class It, class Less>
void parallel_sort(It first, int64_t n, Less less, int64_t min_chunk = 16384) {
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(8, n / min_chunk));
    std::vector<int64_t> cut(static_cast<size_t>(nch) + 1);
    for (int64_t c = 0; c <= nch; ++c) cut[size_t(c)] = n * c / nch;
    parallel_for(nch, [&](int64_t cb, int64_t ce) {
        for (int64_t c = cb; c < ce; ++c) std::sort(first + cut[size_t(c)], first + cut[size_t(c) + 1], less);
    }, 1);
    for (int64_t w = 1; w < nch; w *= 2) {
        std::vector<std::thread> th;
        for (int64_t c = 0; c + w < nch; c += 2 * w) {
            const int64_t lo = cut[size_t(c)], mid = cut[size_t(c + w)], hi = cut[size_t(std::min(nch, c + 2 * w))];
            th.emplace_back([first, &less, lo, mid, hi] { std::inplace_merge(first + lo, first + mid, first + hi, less); });
        }
        for (auto& t : th) t.join();
    }
}

}  // namespace bem

struct bem_ctx {
    int device = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;
    std::vector<bem_tuning> tuning;   // autotuned launch parameters by size class (empty: defaults)
    // streams of destroyed problems, handed to new ones (creating a stream costs about 0.3 ms and
    // destroying one synchronises the device)
    std::mutex stream_mu;
    std::vector<hipStream_t> free_streams;
};

struct bem_problem {
    bem_ctx* ctx = nullptr;
    bem_tuning tune{};                  // launch parameters of this problem (defaults filled in)
    bem::MeshTopo topo;
    int64_t N = 0, ldw = 0, ldI = 0, n_near = 0;
    int64_t panel_rows = 0, n_panels = 0;   // requested rows per pair-matrix panel; panels used
    int64_t panels_replanned = 0;           // 1: the panels were planned again after the sector analysis
    hipStream_t aux_stream = nullptr;   // second stream of the preconditioner set-up (created on first use)
    bool has_w32 = false, has_pairs = false;
    int near_order = 10;
    hipStream_t stream = nullptr;
    bem::DeviceBuffer W64, W32, I;          // W (N x ldw), optional FP32 copy, optional I (nt x ldI)
    bem::DeviceBuffer normal, area;         // per-triangle geometry for the right-hand side
    bem::DeviceBuffer dof_ptr, dof_tri, dof_c;  // dof -> triangle CSR
    bem::DeviceBuffer tri_ptr, tri_dof, tri_corner, tri_c;  // triangle -> dof CSR
    // scratch of the multi-column product: transposed right-hand sides (ldw x 16, FP64-sized),
    // per-split partial sums (16 splits x 16 columns x ldw), and for the symmetric product the
    // super-tile lists ([0] FP32, [1] FP64 matrix) and the block-row partials
    // (ldw / 64 x (mv_nst + 1) x 1024 values).  Calls on one problem must not overlap.
    bem::DeviceBuffer mv_xt, mv_partial, mv_tiles[2], mv_sym;
    int64_t mv_nst[2] = {0, 0}, mv_ntiles[2] = {0, 0};
    int mv_ks[2] = {8, 4};   // super-block edge of the symmetric product ([0] FP32, [1] FP64 matrix)
    // double-layer potential: per-triangle records (normal, Gauss points, n . y) and the 7-point rule,
    // built on the first evaluation
    bem::DeviceBuffer dl_rec, dl_rule;
    double t_assemble = 0, t_host = 0;
    // device times of the assembly phases: bem_assemble returns while the contraction (whole pair
    // matrix) or the panels still run, so their events are kept and read when the information is
    // first asked for
    mutable double t_far = 0, t_near = 0, t_contract = 0;
    mutable hipEvent_t ev_contract[2] = {nullptr, nullptr};
    mutable std::vector<hipEvent_t> ev_spans;   // panels: (far, near, contraction) start/end pairs
    mutable std::mutex info_mu;   // bem_problem_get_info may be called from several threads
    // calls that queue work using the problem's shared scratch (products, solves, preconditioner
    // applications, potentials) take this lock, so two threads calling on one problem serialise
    // instead of interleaving their kernels on its stream
    mutable std::mutex call_mu;
    int64_t bytes = 0;
    // Locality order (triangle meshes): the problem numbers vertices and triangles in Morton order
    // of their positions, so that blocks of consecutive dofs are compact patches; every entry point
    // takes and returns dof-, vertex- and triangle-indexed data in the caller's numbering.
    // vert_user / tri_user: the caller's index of an internal vertex / triangle (tri_int the
    // inverse); dof_user / dof_int: internal dof -> caller's dof and back (also on the device).
    bool renumbered = false;
    std::vector<int32_t> vert_user, tri_user, tri_int, dof_user, dof_int;
    bem::DeviceBuffer d_dof_user, d_dof_int;
};

namespace bem {

// Locality order of a valid triangle mesh (indices in range, finite coordinates): vert_user[i] and
// tri_user[t] are the input indices of the vertex / triangle placed at i / t, sorted by the Morton
// code of the vertex position / triangle centroid (21 bits per axis over the vertices' bounding
// box), ties by index (topology.cpp).
void locality_order(const double* V, int64_t nv, const int32_t* T, int64_t nt, std::vector<int32_t>& vert_user,
                    std::vector<int32_t>& tri_user);
// Device copies of a renumbered mesh from the caller's device copies: Vout[i] = V[vert_user[i]],
// Tout[t] = vert_int(T[tri_user[t]]) (assemble.hip)
void renumber_mesh_device(const double* dV, const int32_t* dT, int64_t nv, int64_t nt, const int32_t* d_vert_user,
                          const int32_t* d_vert_int, const int32_t* d_tri_user, double* Vout, int32_t* Tout, hipStream_t s);
// dst[c][i] = src[c][idx[i]] for i < N, c < k (columns of leading dimensions lds and ldd)
// (solver.hip); with the problem's dof maps it moves vectors between the caller's dof order and
// the internal one
void permute_cols_device(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t N, int k, const int32_t* idx,
                         hipStream_t s);
// out[r][j] = W[rows[r]][cols[j]] (r < nrows, j < ncols; out row-major, ld ncols) (solver.hip)
void gather_rows_device(const double* W, int64_t ldw, const int32_t* d_rows, int64_t nrows, const int32_t* d_cols,
                        int64_t ncols, double* out, hipStream_t s);

// assembly (assemble.hip)
// Assembles W for the mesh (V, T).  analyse(near) runs on the host while the far-field pass is on
// the device: it must fill p->topo (and the near list) or throw the mesh's validation error.
// dV, dT: optional device copies of V and T, which the kernels then read instead of an upload.
void assemble_device(bem_problem* p, const double* V, int64_t nv, const int32_t* T, int64_t nt,
                     const std::function<void(NearList&)>& analyse, const double* dV = nullptr,
                     const int32_t* dT = nullptr);
void rhs_device(const bem_problem* p, const double* d_g, int k, double* d_L, hipStream_t s);
// two-dimensional variant (twod.hip): analyses the segment mesh into p->topo and assembles W
void assemble_2d_device(bem_problem* p, const double* V2, int64_t nv, const int32_t* S, int64_t ns);
void jump_values_device(const bem_problem* p, const double* d_phi, double* d_jump, hipStream_t s);
// double-layer potential (potential.hip): U [k][m] at targets X [m][3] for phi [k][N], all on the device
void double_layer_device(bem_problem* p, const double* d_phi, int k, const double* d_X, int64_t m, double* d_U,
                         hipStream_t s);

// a non-blocking stream of the context's device: a released one, or a new one
hipStream_t acquire_stream(bem_ctx* c);
// gives back a stream with no queued work (the caller has synchronised it)
void release_stream(bem_ctx* c, hipStream_t s);

// Default refresh factor of the mixed-precision PCG's residual replacement: about the square root
// of the FP32 unit roundoff (2^-24), so that between two replacements the recurrence residual falls
// no further than the FP32 products' rounding lets it follow the true residual.
constexpr double kRefreshDefault = 2.5e-4;

// dense products (solver.hip); x, y column-major [k][N] with leading dimension ldx
void matvec_setup(bem_problem* p, hipStream_t s);   // after W is allocated (ldw set)
// gate != nullptr: a device word; the product's kernels do nothing while it is 0 (y keeps its values)
void matvec_device(const bem_problem* p, bool fp32, const double* d_x, int64_t ldx, int k,
                   double* d_y, hipStream_t s, const int* gate = nullptr);
// Continuous batching of a block PCG (serving loop): a fixed number of column slots, each running
// its own CG (per-column scalars and tolerance).  At every check point the solver reports the
// columns that have stopped since the last one and asks for new columns to start in the free slots.
struct PcgColumnResult {
    int iters = 0, status = BEM_OK, refreshes = 0;
    double relres = 0.0;
};
struct PcgNewColumn {
    int slot;
    double g[3];      // constant Neumann data of the column (its right-hand side is built on the device)
    double tol;       // relative residual tolerance
};
struct PcgSlots {
    // column `slot` has stopped (converged, broken down, or out of iterations); d_x is its solution
    // on the device, final once the solver's stream is synchronised (it is, at this call)
    std::function<void(int slot, const double* d_x, const PcgColumnResult& r)> finished;
    // the free slots and the number of columns still running -> the columns to start now.  When it
    // returns none while no column is running, the batch ends.
    std::function<void(const std::vector<int>& free_slots, int running, std::vector<PcgNewColumn>& start)> admit;
    bool graphed = false;   // out: the iterations ran as graph replays
};
// runs the block PCG on `slots` column slots until the hooks stop admitting; max_iter per column
void pcg_serve(bem_problem* p, const bem_precond* M, bool mixed, int slots, int max_iter, int check_every,
               PcgSlots& hooks);

// the same products with their scratch in the device array of bem_matvec_noalloc (solver.hip):
// its size, the per-device address (looked up once per device, with that device current), the
// bytes one product of this problem needs there, and the launch
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;
void* noalloc_scratch_address(int device);
size_t noalloc_matvec_bytes(const bem_problem* p, bool fp32, int k);
void matvec_device_noalloc(const bem_problem* p, bool fp32, const double* d_x, int64_t ldx, int k, double* d_y,
                           hipStream_t s, void* scratch);

}  // namespace bem

// ------------------------------------------------------------------------------------------
// Preconditioner (precond.hip)
// ------------------------------------------------------------------------------------------
struct bem_precond {
    bem_problem* p = nullptr;
    bool fp32 = false, use_coarse = true;
    int64_t nblocks = 0, n_faces = 0, n_wb = 0, nH = 0, max_face = 0;
    std::vector<int64_t> blk_n, blk_npad, blk_idx_off, blk_mat_off;
    int64_t idx_total = 0, mat_total = 0;
    bem::DeviceBuffer idx;          // concatenated dof indices of the blocks (int32)
    bem::DeviceBuffer blk_meta;     // per block: n, npad, idx_off, mat_off (int64 x 4)
    bem::DeviceBuffer inv64, inv32; // explicit block inverses, npad x npad row-major each
    bem::DeviceBuffer tasks;        // apply tasks: (block, row0, nrows, 0) as int4
    int64_t ntasks = 0, max_npad = 0, xg_rows = 0;
    bem::DeviceBuffer xg;           // apply scratch: gathered, transposed block right-hand sides
    // coarse space: R_H as CSR over coarse dofs and over fine dofs, and (R_H W R_H^T)^{-1}
    bem::DeviceBuffer rh_ptr, rh_col, rh_val, rht_ptr, rht_row, rht_val, WHinv;
    // diagonal wire basket: its dofs and 1 / W_dd (then the wire basket is not one of the blocks)
    bool wb_diag = false;
    bem::DeviceBuffer wb_idx, wb_dinv;
    double diag_shift = 0.0;        // sigma added to the diagonal of every block before factorising
    int64_t bytes = 0;
    double t_setup = 0;
};

namespace bem {
// Host construction of the dof classes and R_H, then device factorisation (precond.hip).
void precond_setup_device(bem_precond* m, const int32_t* patch_of_triangle, const double* cV, int64_t ncv,
                          const int32_t* cT, int64_t nct, const int32_t* coarse_of_triangle);
// z = M r for k columns (column-major, leading dimension ld); fp32 selects the FP32 inverses.
void precond_apply_device(const bem_precond* m, bool fp32, const double* r, int64_t ld, int k, double* z,
                          hipStream_t s, double* coarse_scratch);
// scratch (doubles) needed by precond_apply_device for k columns
int64_t precond_scratch_size(const bem_precond* m, int k);
}  // namespace bem
