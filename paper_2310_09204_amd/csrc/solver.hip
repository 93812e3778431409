// Preconditioned conjugate gradients for W Phi = L (paper: Remark "Bound on the number of
// Preconditioned Conjugate Gradient iterations" -- PCG on P_ad = M A_h; x0 = 0; the stopping rule
// ||L - W x||_2 <= tol ||L||_2 on the unpreconditioned residual is the build's choice).
//
// k right-hand sides run side by side: each iteration streams W once for all columns (row-panel
// matvec), and every column keeps its own scalars (alpha, beta, r.z) in device memory, so an
// iteration is a fixed sequence of kernels with no host round trip.  That sequence is captured
// once into a hipGraph and replayed; the host only reads the per-column status every few
// iterations.  Converged columns are frozen (their updates become no-ops), so iteration counts are
// exact.  The mixed-precision mode is iterative refinement: residuals with the FP64 matrix, each
// correction from a PCG on the FP32 copy of W with FP32 block inverses (FP64 dot products, vector
// updates and coarse solve).
#include <algorithm>
#include <chrono>
#include <cmath>

#include "internal.h"
#include "strips.h"
#include <type_traits>

namespace bem {

namespace {

// Per-column scalars of the block (P)CG, kept on the device.  `due` marks a column of the
// mixed-precision iteration that asks for a residual replacement in the current iteration;
// `refreshes` counts the column's replacements; rr_ref is r.r of its last true residual.
struct ColState {
    double rz, pq, rr, alpha, beta, bb, tol2, rr_ref;
    int active, iters, flag, due, refreshes, pad2;
};

constexpr int kStatBreakdown = 2;

// ---------------------------------------------------------------------------------------------
// dense row-panel matvec: one wave per row, 16-byte loads of W, k columns
// ---------------------------------------------------------------------------------------------
template <typename MT, typename AT, int K>
__global__ __launch_bounds__(256) void k_matvec(const MT* __restrict__ W, int64_t ldw, int64_t N,
                                                const double* __restrict__ x, int64_t ldx, int kc,
                                                double* __restrict__ y, int64_t ldy, const int* __restrict__ gate) {
    if (gate && !*gate) return;
    const int lane = threadIdx.x & 63;
    const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (row >= N) return;
    constexpr int VEC = 16 / sizeof(MT);
    const MT* w = W + row * ldw;
    AT acc[K];
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = AT(0);
    const int64_t step = 64 * VEC;
    const int64_t nfull = (N / step) * step;
    for (int64_t j = int64_t(lane) * VEC; j < nfull; j += step) {
        MT wv[VEC];
        if constexpr (VEC == 2) {
            const double2 t = *reinterpret_cast<const double2*>(w + j);
            wv[0] = t.x; wv[1] = t.y;
        } else {
            const float4 t = *reinterpret_cast<const float4*>(w + j);
            wv[0] = t.x; wv[1] = t.y; wv[2] = t.z; wv[3] = t.w;
        }
#pragma unroll
        for (int c = 0; c < K; ++c) {
            if (c >= kc) break;
            const double* xc = x + int64_t(c) * ldx + j;
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[c] = fma(AT(wv[v]), AT(xc[v]), acc[c]);
        }
    }
    for (int64_t j = nfull + lane; j < N; j += 64) {
        const AT wj = AT(w[j]);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            if (c >= kc) break;
            acc[c] = fma(wj, AT(x[int64_t(c) * ldx + j]), acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
        AT v = acc[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        acc[c] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (c < kc) y[int64_t(c) * ldy + row] = double(acc[c]);
    }
}

// ---------------------------------------------------------------------------------------------
// multi-column product Y = W X on the matrix cores (the strip routine in strips.h is shared with
// the preconditioner apply): each wave owns a 16-row strip of W and a column range; X is
// transposed once per product into Xt[j][16] so every B fragment is one coalesced read per 16 lanes.
// ---------------------------------------------------------------------------------------------
template <typename MT>
__global__ void k_transpose_x(const double* __restrict__ x, int64_t ldx, int kc, int64_t N, int64_t rows,
                              MT* __restrict__ xt, const int* __restrict__ gate) {
    if (gate && !*gate) return;
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= rows * 16) return;
    const int64_t j = e >> 4;
    const int n = int(e & 15);
    xt[e] = (n < kc && j < N) ? MT(x[int64_t(n) * ldx + j]) : MT(0);
}

// Y = W X for up to 16 columns on the matrix cores.  A block owns 64 rows of W and a range of
// columns (split-K over blockIdx.y).  Per tile of TC columns (256 bytes of each row), every wave
// loads 16 of the 64 rows with 16 lanes on one row's contiguous 256 bytes, so each load
// instruction reads four whole row segments; the tile and the matching X tile (TC x 16, from the
// transposed right-hand sides) go to LDS, and wave w then runs the TC/4 MFMAs of rows 16w .. 16w+15
// from LDS.  Two LDS buffers: the next tile's loads are in flight while the current one is used,
// one barrier per tile.  Results go to y directly (one split) or to per-split partial sums.
template <typename MT>
__global__ __launch_bounds__(256) void k_matvec_mfma(const MT* __restrict__ W, int64_t ldw, int64_t N,
                                                     const MT* __restrict__ xt, int64_t cols_per_split, int kc,
                                                     double* __restrict__ y, int64_t ldy, double* __restrict__ partial,
                                                     const int* __restrict__ gate) {
    if (gate && !*gate) return;
    using MC = MatrixCore<MT>;
    using V16 = typename std::conditional<sizeof(MT) == 4, float4, double2>::type;
    constexpr int VEC = 16 / sizeof(MT);
    constexpr int TC = 256 / sizeof(MT);
    __shared__ MT tA[2][64][TC + VEC];
    __shared__ MT tX[2][TC * 16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = lane & 15, kg = lane >> 4;
    const int64_t row0 = int64_t(blockIdx.x) * 64;
    const int split = blockIdx.y;
    const int64_t c0 = int64_t(split) * cols_per_split;
    const int64_t c1 = min<int64_t>(ldw, c0 + cols_per_split);
    const int lr = tid >> 4;           // row of a 16-row load group
    const int lc = (tid & 15) * VEC;   // column within the tile
    typename MC::V acc = {0, 0, 0, 0};
    // FP32 matrices: the matrix-core sums run over at most kFlushTiles tiles (1024 columns) and are
    // then added into FP64, so the rounding of long rows (N ~ 1e5) stays at the level of one chunk
    constexpr int kFlushTiles = 1024 / TC;
    double acc64[4] = {0.0, 0.0, 0.0, 0.0};
    int since_flush = 0;
    V16 va[4], vx;
    auto fetch = [&](int64_t jc) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = row0 + q * 16 + lr;
            if (row < N) va[q] = *reinterpret_cast<const V16*>(W + row * ldw + jc + lc);
            else va[q] = V16{};
        }
        vx = reinterpret_cast<const V16*>(xt + jc * 16)[tid];
    };
    if (c0 < c1) fetch(c0);
    int buf = 0;
    for (int64_t jc = c0; jc < c1; jc += TC) {
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<V16*>(&tA[buf][q * 16 + lr][lc]) = va[q];
        reinterpret_cast<V16*>(&tX[buf][0])[tid] = vx;
        __syncthreads();
        if (jc + TC < c1) fetch(jc + TC);
#pragma unroll
        for (int st = 0; st < TC / 4; ++st)
            acc = MC::mac(tA[buf][wave * 16 + i][4 * st + kg], tX[buf][(4 * st + kg) * 16 + i], acc);
        buf ^= 1;
        if constexpr (sizeof(MT) == 4) {
            if (++since_flush == kFlushTiles) {
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[r] += double(acc[r]);
                acc = typename MC::V{0, 0, 0, 0};
                since_flush = 0;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[r] += double(acc[r]);
    if (i < kc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t rr = row0 + wave * 16 + MC::out_row(kg, r);
            if (rr < N) {
                if (partial) partial[(int64_t(split) * 16 + i) * ldw + rr] = acc64[r];
                else y[int64_t(i) * ldy + rr] = acc64[r];
            }
        }
    }
}

// Symmetric product Y = W X for up to 16 columns that reads only the upper half of W (the Galerkin
// matrix of a symmetric bilinear form is symmetric).  The 64-row blocks are grouped into super-blocks
// of KS (a launch parameter); a workgroup takes one super-tile (I, J), I <= J, and walks it column by
// column (on a diagonal super-tile only the blocks on and above the diagonal).  Each 64 x 64 block
// is read from HBM once and used twice:
//  * rows of bi, W_bi,bj X_bj: through LDS as in the plain product (wave w: rows 16w .. 16w+15);
//  * rows of bj, W_bi,bj^T X_bi (bi < bj): straight from the registers of the coalesced load.  Lane
//    16 kg + j holds VEC consecutive columns of row r(kg); with the row as the summation index (k
//    slot kg) and the column as the output index (lane j) every loaded vector feeds VEC matrix-core
//    products, one per class of output columns.  Each wave sums over its own 16 rows of the block;
//    the four wave sums are added through LDS once per block column.
// Row sums of the super-tile's block rows are kept in LDS (one accumulator fragment per thread and
// block row, carried through the matrix cores block after block) and column sums in registers,
// each over at most KS * 64 products; each leaves once as a partial of its block row, in MT (exact
// for FP32 accumulators).  k_symv_reduce adds the nst + 1 partials of each block row in FP64 in a
// fixed order.  HBM traffic: half of W plus 1/KS of it in partials, written and read back.
// KS is a launch parameter chosen by the autotuner: 2, 4 or 8 blocks for the FP64 matrix (default
// 4), 4, 8 or 16 for the FP32 copy (default 8).
template <typename MT, int KS>
__global__ __launch_bounds__(256) void k_symv_mfma(const MT* __restrict__ W, int64_t ldw, int64_t N, const MT* __restrict__ xt,
                                                   int64_t nb, int64_t nst, const int2* __restrict__ tiles,
                                                   MT* __restrict__ part, const int* __restrict__ gate) {
    if (gate && !*gate) return;
    using MC = MatrixCore<MT>;
    using V = typename MC::V;
    using V16 = typename std::conditional<sizeof(MT) == 4, float4, double2>::type;
    constexpr int VEC = 16 / sizeof(MT);
    constexpr int HV = 64 / (16 * VEC);   // 16-lane segments per 64-column block row
    constexpr int NL = 4 * HV * VEC;      // values of one block held by a thread
    __shared__ MT tA[64][64 + VEC];
    __shared__ V accl[KS][256];
    const int2 tile = tiles[blockIdx.x];
    const int64_t I = tile.x, J = tile.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i = lane & 15, kg = lane >> 4;
    const int64_t bi0 = I * KS, bi1 = min<int64_t>(nb, bi0 + KS);
    const int64_t bj0 = J * KS, bj1 = min<int64_t>(nb, bj0 + KS);
#pragma unroll
    for (int p = 0; p < KS; ++p) accl[p][tid] = V{0, 0, 0, 0};   // own slots: no barrier needed
    // thread (w, kg, i) loads rows 16 q + 4 w + kg (q < 4), columns 16 VEC h + VEC i .. + VEC - 1 (h < HV)
    MT a[NL], xc[4];
    auto fetch = [&](int64_t bi, int64_t bj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = bi * 64 + 16 * q + 4 * w + kg;
#pragma unroll
            for (int h = 0; h < HV; ++h) {
                V16 v{};
                if (row < N) v = *reinterpret_cast<const V16*>(W + row * ldw + bj * 64 + 16 * VEC * h + VEC * i);
                MT* d = a + (q * HV + h) * VEC;
                if constexpr (VEC == 4) { d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w; }
                else { d[0] = v.x; d[1] = v.y; }
            }
            xc[q] = xt[row * 16 + i];
        }
    };
    fetch(bi0, bj0);
    for (int64_t bj = bj0; bj < bj1; ++bj) {
        MT xr[16];   // X_bj as the B operand of the row product
#pragma unroll
        for (int st = 0; st < 16; ++st) xr[st] = xt[(bj * 64 + 4 * st + kg) * 16 + i];
        V accc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) accc[t] = V{0, 0, 0, 0};
        const int64_t last = I == J ? bj : bi1 - 1;
        for (int64_t bi = bi0; bi <= last; ++bi) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int h = 0; h < HV; ++h) {
                    const MT* d = a + (q * HV + h) * VEC;
                    V16 v;
                    if constexpr (VEC == 4) v = V16{d[0], d[1], d[2], d[3]};
                    else v = V16{d[0], d[1]};
                    *reinterpret_cast<V16*>(&tA[16 * q + 4 * w + kg][16 * VEC * h + VEC * i]) = v;
                }
            __syncthreads();
            if (bi != bj) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int t = 0; t < 4; ++t) accc[t] = MC::mac(xc[q], a[(q * HV + t / VEC) * VEC + t % VEC], accc[t]);
            }
            // the next block in flight while this one's row product runs
            if (bi < last) fetch(bi + 1, bj);
            else if (bj + 1 < bj1) fetch(bi0, bj + 1);
            V acc = accl[bi - bi0][tid];
#pragma unroll
            for (int st = 0; st < 16; ++st) acc = MC::mac(tA[16 * w + i][4 * st + kg], xr[st], acc);
            accl[bi - bi0][tid] = acc;
            __syncthreads();
        }
        // column partial of block column bj: the four waves' sums, through the tile's LDS
        MT* red = &tA[0][0];   // [wave][16 right-hand sides][64 columns]
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                red[(w * 16 + MC::out_row(kg, r)) * 64 + 16 * VEC * (t / VEC) + VEC * i + t % VEC] = accc[t][r];
        __syncthreads();
        MT* dst = part + (bj * (nst + 1) + (nst - bj / KS) + I) * 1024;
#pragma unroll
        for (int o = tid; o < 1024; o += 256) dst[o] = (red[o] + red[1024 + o]) + (red[2048 + o] + red[3072 + o]);
        __syncthreads();
    }
    // row partials of the super-tile's block rows
    for (int64_t bi = bi0; bi < bi1; ++bi) {
        MT* dst = part + (bi * (nst + 1) + (J - bi / KS)) * 1024;
        const V acc = accl[bi - bi0][tid];
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[i * 64 + 16 * w + MC::out_row(kg, r)] = acc[r];
    }
}

// y[c][e] = the nst + 1 partials of block row b = e / 64 added in FP64: row partials J = b / KS ..
// nst - 1, then column partials I = 0 .. b / KS (slot order; loads issued eight at a time)
template <typename MT>
__global__ void k_symv_reduce(const MT* __restrict__ part, int64_t nst, int64_t N, double* __restrict__ y, int64_t ldy,
                              const int* __restrict__ gate) {
    if (gate && !*gate) return;
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= N) return;
    const MT* p = part + (e >> 6) * (nst + 1) * 1024 + c * 64 + (e & 63);
    double s = 0.0;
    int64_t q = 0;
    for (; q + 8 <= nst + 1; q += 8) {
        MT v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(q + u) * 1024];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += double(v[u]);
    }
    for (; q <= nst; ++q) s += double(p[q * 1024]);
    y[int64_t(c) * ldy + e] = s;
}

__global__ void k_reduce_splits(const double* __restrict__ partial, int S, int kc, int64_t N, int64_t ldw,
                                double* __restrict__ y, int64_t ldy, const int* __restrict__ gate) {
    if (gate && !*gate) return;
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= int64_t(kc) * N) return;
    const int n = int(e / N);
    const int64_t r = e % N;
    double s = 0.0;
    for (int q = 0; q < S; ++q) s += partial[(int64_t(q) * 16 + n) * ldw + r];
    y[int64_t(n) * ldy + r] = s;
}

// ---------------------------------------------------------------------------------------------
// vector kernels (grid: G blocks x k columns; block-partial sums reduced in a fixed order)
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[4];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t ld, int64_t N, double* __restrict__ partial) {
    const int c = blockIdx.y;
    const double* ac = a + int64_t(c) * ld;
    const double* bc = b + int64_t(c) * ld;
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256) s = fma(ac[i], bc[i], s);
    s = block_sum(s);
    if (threadIdx.x == 0) partial[int64_t(c) * gridDim.x + blockIdx.x] = s;
}

__device__ __forceinline__ double reduce_partials(const double* __restrict__ p, int G) {
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) s += p[i];
    return block_sum(s);
}

// p.q -> alpha
__global__ __launch_bounds__(256) void k_alpha(const double* __restrict__ partial, int G, ColState* __restrict__ st,
                                               double* __restrict__ hist, int max_hist) {
    const int c = blockIdx.x;
    const double pq = reduce_partials(partial + int64_t(c) * G, G);
    if (threadIdx.x == 0) {
        ColState& s = st[c];
        s.pq = pq;
        if (s.active) {
            if (!(pq > 0.0) || !isfinite(pq)) {
                s.active = 0;
                s.flag = kStatBreakdown;
                s.alpha = 0.0;
            } else {
                s.alpha = s.rz / pq;
                if (s.iters < max_hist) hist[int64_t(c) * 2 * max_hist + s.iters] = s.alpha;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_update_xr(double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   int64_t ld, int64_t N, const ColState* __restrict__ st,
                                                   double* __restrict__ partial) {
    const int c = blockIdx.y;
    const ColState& s = st[c];
    double acc = 0.0;
    if (s.active) {
        const double al = s.alpha;
        double* xc = x + int64_t(c) * ld;
        double* rc = r + int64_t(c) * ld;
        const double* pc = p + int64_t(c) * ld;
        const double* qc = q + int64_t(c) * ld;
        for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256) {
            xc[i] = fma(al, pc[i], xc[i]);
            const double ri = fma(-al, qc[i], rc[i]);
            rc[i] = ri;
            acc = fma(ri, ri, acc);
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[int64_t(c) * gridDim.x + blockIdx.x] = acc;
}

// Mixed precision, after the update of x and r: a column is due for residual replacement in this
// iteration when its recurrence r.r has met the tolerance (convergence is judged on true residuals
// only) or has fallen by refresh2 since its last true residual (so that the FP32 products'
// rounding never dominates the recurrence).
__global__ __launch_bounds__(256) void k_check_due(const double* __restrict__ partial, int G, ColState* __restrict__ st,
                                                   double refresh2) {
    const int c = blockIdx.x;
    const double rr = reduce_partials(partial + int64_t(c) * G, G);
    if (threadIdx.x == 0) {
        ColState& s = st[c];
        s.due = (s.active && (!(rr > s.tol2 * s.bb) || rr < refresh2 * s.rr_ref)) ? 1 : 0;
    }
}

// gate[which] = 1 if any column is active (which = 0) or due (which = 1): the product kernels that
// take the gate do nothing when it is 0, so that a captured iteration costs little once every
// column has stopped, and the FP64 product of a replacement runs only when a column is due.  That
// product covers the whole block, so every active column is replaced with the due ones: the columns
// share one replacement schedule and one FP64 product per replacement.
__global__ __launch_bounds__(256) void k_gate(const ColState* __restrict__ st, int k, int which, int* __restrict__ gate) {
    int any = 0;
    for (int c = threadIdx.x; c < k; c += 256) any |= which ? st[c].due : st[c].active;
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) gate[which] = any ? 1 : 0;
}

// r.r from block partials; it is the true residual of x in the FP64 iteration and in a mixed one
// with replacement (gate[1]), and only a true residual decides convergence.
__global__ __launch_bounds__(256) void k_check(const double* __restrict__ partial, int G, ColState* __restrict__ st,
                                               int mixed, const int* __restrict__ gate) {
    const int c = blockIdx.x;
    const double rr = reduce_partials(partial + int64_t(c) * G, G);
    if (threadIdx.x == 0) {
        ColState& s = st[c];
        if (s.active) {
            s.iters += 1;
            s.rr = rr;
            const bool replaced = mixed && gate[1];
            const bool true_res = !mixed || replaced;
            s.due = 0;
            if (replaced) {
                s.refreshes += 1;
                s.rr_ref = rr;
            }
            if (!isfinite(rr)) {
                s.active = 0;
                s.flag = kStatBreakdown;
            } else if (true_res && rr <= s.tol2 * s.bb) {
                s.active = 0;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_beta(const double* __restrict__ partial, int G, ColState* __restrict__ st,
                                              double* __restrict__ hist, int max_hist) {
    const int c = blockIdx.x;
    const double rz = reduce_partials(partial + int64_t(c) * G, G);
    if (threadIdx.x == 0) {
        ColState& s = st[c];
        if (s.active) {
            s.beta = rz / s.rz;
            s.rz = rz;
            const int it = s.iters - 1;
            if (it < max_hist) hist[int64_t(c) * 2 * max_hist + max_hist + it] = s.beta;
        }
    }
}

__global__ __launch_bounds__(256) void k_update_p(double* __restrict__ p, const double* __restrict__ z, int64_t ld,
                                                  int64_t N, const ColState* __restrict__ st) {
    const int c = blockIdx.y;
    const ColState& s = st[c];
    if (!s.active) return;
    const double be = s.beta;
    double* pc = p + int64_t(c) * ld;
    const double* zc = z + int64_t(c) * ld;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256) pc[i] = fma(be, pc[i], zc[i]);
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t ld, int64_t N) {
    const int c = blockIdx.y;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256)
        b[int64_t(c) * ld + i] = a[int64_t(c) * ld + i];
}

__global__ void k_fill(double* __restrict__ a, double v, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) a[i] = v;
}

// r = b - y
__global__ void k_residual(const double* __restrict__ b, const double* __restrict__ y, double* __restrict__ r,
                           int64_t ld, int64_t N) {
    const int c = blockIdx.y;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256)
        r[int64_t(c) * ld + i] = b[int64_t(c) * ld + i] - y[int64_t(c) * ld + i];
}

// when some column is due (gate[1]): r = b - y for every active column, with the partial sums of
// r.r (as k_update_xr leaves them)
__global__ __launch_bounds__(256) void k_residual_due(const double* __restrict__ b, const double* __restrict__ y,
                                                      double* __restrict__ r, int64_t ld, int64_t N,
                                                      const ColState* __restrict__ st, double* __restrict__ partial,
                                                      const int* __restrict__ gate) {
    const int c = blockIdx.y;
    if (!gate[1] || !st[c].active) return;
    double acc = 0.0;
    {
        const double* bc = b + int64_t(c) * ld;
        const double* yc = y + int64_t(c) * ld;
        double* rc = r + int64_t(c) * ld;
        for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256) {
            const double ri = bc[i] - yc[i];
            rc[i] = ri;
            acc = fma(ri, ri, acc);
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[int64_t(c) * gridDim.x + blockIdx.x] = acc;
}

__global__ void k_axpy_cols(double* __restrict__ x, const double* __restrict__ d, int64_t ld, int64_t N) {
    const int c = blockIdx.y;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256)
        x[int64_t(c) * ld + i] += d[int64_t(c) * ld + i];
}

// a serving column that ran out of iterations stops (its state is kept for the report)
__global__ void k_stop_column(ColState* __restrict__ st) { st->active = 0; }

// state init from partials of b.b, r.r, r.z
__global__ __launch_bounds__(256) void k_init_state(const double* __restrict__ pbb, const double* __restrict__ prr,
                                                    const double* __restrict__ prz, int G, const double* __restrict__ tol2,
                                                    ColState* __restrict__ st) {
    const int c = blockIdx.x;
    const double bb = reduce_partials(pbb + int64_t(c) * G, G);
    const double rr = reduce_partials(prr + int64_t(c) * G, G);
    const double rz = reduce_partials(prz + int64_t(c) * G, G);
    if (threadIdx.x == 0) {
        ColState s{};
        s.bb = bb;
        s.rr = rr;
        s.rz = rz;
        s.tol2 = tol2[c];
        s.rr_ref = rr;
        s.iters = 0;
        s.flag = 0;
        s.due = 0;
        s.refreshes = 0;
        if (!isfinite(bb) || !isfinite(rr) || !isfinite(rz)) {
            s.active = 0;
            s.flag = kStatBreakdown;
        } else {
            s.active = (bb > 0.0 && rr > s.tol2 * bb) ? 1 : 0;
        }
        st[c] = s;
    }
}

inline unsigned gblocks(int64_t N) { return unsigned(std::max<int64_t>(1, std::min<int64_t>(1024, (N + 255) / 256))); }

// out[r][j] = W[rows[r]][cols[j]]
__global__ void k_gather_rows(const double* __restrict__ W, int64_t ldw, const int32_t* __restrict__ rows,
                              const int32_t* __restrict__ cols, int64_t ncols, double* __restrict__ out) {
    const int64_t r = blockIdx.y;
    const double* wr = W + int64_t(rows[r]) * ldw;
    for (int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x; j < ncols; j += int64_t(gridDim.x) * 256)
        out[r * ncols + j] = wr[cols[j]];
}

// dst[c][i] = src[c][idx[i]]
__global__ void k_permute_cols(const double* __restrict__ src, int64_t lds, double* __restrict__ dst, int64_t ldd,
                               int64_t N, const int32_t* __restrict__ idx) {
    const int c = blockIdx.y;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256)
        dst[int64_t(c) * ldd + i] = src[int64_t(c) * lds + idx[i]];
}

// xt: transposed right-hand sides (ldw x 16 of MT); part: split partials of the plain product
// (16 x 16 x ldw doubles); sp: block-row partials of the symmetric product (ldw / 64 x (nst + 1) x
// 1024 of MT).  Every entry of the three that a later kernel reads is written first, each call.
template <typename MT, typename AT>
void launch_matvec(const bem_problem* p, const MT* W, const double* x, int64_t ldx, int k, double* y, int64_t ldy,
                   hipStream_t s, MT* xt, double* part, MT* sp, const int* gate) {
    const int64_t N = p->N, ldw = p->ldw;
    for (int c0 = 0; c0 < k; c0 += 16) {
        const int kc = std::min(16, k - c0);
        const double* xc = x + int64_t(c0) * ldx;
        double* yc = y + int64_t(c0) * ldy;
        const int ty = sizeof(MT) == 4 ? 0 : 1;
        if (kc == 1 && p->mv_ntiles[ty] == 0) {
            // one column of a one-block matrix: a plain streaming dot product per row (one wave per row)
            hipLaunchKernelGGL((k_matvec<MT, AT, 1>), dim3(unsigned((N + 3) / 4)), dim3(256), 0, s, W, ldw, N, xc, ldx, kc, yc, ldy, gate);
            HIP_CHECK(hipGetLastError());
            continue;
        }
        hipLaunchKernelGGL(k_transpose_x<MT>, dim3(unsigned((ldw * 16 + 255) / 256)), dim3(256), 0, s, xc, ldx, kc, N, ldw, xt, gate);
        if (p->mv_ntiles[ty] > 0) {
            // W is symmetric: read its upper half once and apply every block to both sides (also
            // for a single column: half the bytes outweigh the idle matrix-core columns)
            const dim3 grid(unsigned(p->mv_ntiles[ty])), blk(256);
            const int64_t nbk = ldw / 64, nst = p->mv_nst[ty];
            const int2* tl = p->mv_tiles[ty].as<int2>();
            if constexpr (sizeof(MT) == 4) {
                switch (p->mv_ks[ty]) {
                    case 4: hipLaunchKernelGGL((k_symv_mfma<MT, 4>), grid, blk, 0, s, W, ldw, N, xt, nbk, nst, tl, sp, gate); break;
                    case 16: hipLaunchKernelGGL((k_symv_mfma<MT, 16>), grid, blk, 0, s, W, ldw, N, xt, nbk, nst, tl, sp, gate); break;
                    default: hipLaunchKernelGGL((k_symv_mfma<MT, 8>), grid, blk, 0, s, W, ldw, N, xt, nbk, nst, tl, sp, gate); break;
                }
            } else {
                switch (p->mv_ks[ty]) {
                    case 2: hipLaunchKernelGGL((k_symv_mfma<MT, 2>), grid, blk, 0, s, W, ldw, N, xt, nbk, nst, tl, sp, gate); break;
                    case 8: hipLaunchKernelGGL((k_symv_mfma<MT, 8>), grid, blk, 0, s, W, ldw, N, xt, nbk, nst, tl, sp, gate); break;
                    default: hipLaunchKernelGGL((k_symv_mfma<MT, 4>), grid, blk, 0, s, W, ldw, N, xt, nbk, nst, tl, sp, gate); break;
                }
            }
            hipLaunchKernelGGL(k_symv_reduce<MT>, dim3(unsigned((N + 255) / 256), unsigned(kc)), dim3(256), 0, s, sp,
                               p->mv_nst[ty], N, yc, ldy, gate);
            HIP_CHECK(hipGetLastError());
            continue;
        }
        // split the columns when there are too few 64-row blocks to keep every CU streaming
        const int64_t blocks = (N + 63) / 64;
        int S = 1;
        if (blocks < 1500) {
            S = 4;
            while (S < kMaxSplits && blocks * S < 3000) S *= 2;
        }
        const int64_t quantum = 256 / int64_t(sizeof(MT));   // one LDS tile of columns
        const int64_t cps = ((ldw + S - 1) / S + quantum - 1) / quantum * quantum;
        S = int((ldw + cps - 1) / cps);
        const dim3 grid{unsigned(blocks), unsigned(S), 1u};
        hipLaunchKernelGGL(k_matvec_mfma<MT>, grid, dim3(256), 0, s, W, ldw, N, xt, cps, kc, yc, ldy, S > 1 ? part : nullptr, gate);
        if (S > 1)
            hipLaunchKernelGGL(k_reduce_splits, dim3(unsigned((int64_t(kc) * N + 255) / 256)), dim3(256), 0, s, part, S, kc, N,
                               ldw, yc, ldy, gate);
        HIP_CHECK(hipGetLastError());
    }
}

// smallest / largest eigenvalue of a symmetric tridiagonal matrix by Sturm-sequence bisection
double tridiag_extreme(const std::vector<double>& d, const std::vector<double>& e, bool largest) {
    const int m = int(d.size());
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
        double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    auto count_below = [&](double x) {
        int cnt = 0;
        double q = 1.0;
        for (int i = 0; i < m; ++i) {
            double off = (i > 0) ? e[i - 1] * e[i - 1] : 0.0;
            q = d[i] - x - (i > 0 ? off / q : 0.0);
            if (q == 0.0) q = -1e-300;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    const int target = largest ? m - 1 : 0;
    for (int it = 0; it < 200 && hi - lo > 1e-14 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        double mid = 0.5 * (lo + hi);
        if (count_below(mid) > target) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

double lanczos_condition(const double* alpha, const double* beta, int m) {
    if (m <= 0) return std::nan("");
    std::vector<double> d(m), e(std::max(0, m - 1));
    for (int j = 0; j < m; ++j) {
        d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
        if (j + 1 < m) e[j] = std::sqrt(std::max(0.0, beta[j])) / alpha[j];
    }
    const double lmin = tridiag_extreme(d, e, false), lmax = tridiag_extreme(d, e, true);
    return lmax / lmin;
}

}  // namespace

// scratch of the multi-column products, sized for the problem: transposed right-hand sides, split
// partials of the plain product, and per matrix type the super-tile list of the symmetric product
// and its block-row partials (one buffer, sized for the larger of the two)
void matvec_setup(bem_problem* p, hipStream_t s) {
    p->mv_xt = DeviceBuffer(sizeof(double) * 16 * p->ldw, s);
    p->mv_partial = DeviceBuffer(sizeof(double) * 16 * 16 * p->ldw, s);
    const int64_t nb = p->ldw / 64;
    if (nb < 2) return;   // one block: the plain product
    std::vector<int2> tiles[2];
    size_t sym_bytes = 0;
    for (int ty = 0; ty < 2; ++ty) {
        const int64_t ks = ty == 0 ? p->tune.symv_blocks_fp32 : p->tune.symv_blocks_fp64;
        p->mv_ks[ty] = int(ks);
        const int64_t nst = (nb + ks - 1) / ks;
        // off-diagonal super-tiles first: the half-size diagonal ones fill the tail of the launch
        for (int64_t I = 0; I < nst; ++I)
            for (int64_t J = I + 1; J < nst; ++J) tiles[ty].push_back(int2{int(I), int(J)});
        for (int64_t I = 0; I < nst; ++I) tiles[ty].push_back(int2{int(I), int(I)});
        p->mv_tiles[ty] = upload(tiles[ty], s);
        p->mv_nst[ty] = nst;
        sym_bytes = std::max(sym_bytes, size_t(nb * (nst + 1) * 1024) * (ty == 0 ? sizeof(float) : sizeof(double)));
    }
    p->mv_sym = DeviceBuffer(sym_bytes, s);
    HIP_CHECK(hipStreamSynchronize(s));   // the host lists must outlive their uploads
    for (int ty = 0; ty < 2; ++ty) p->mv_ntiles[ty] = int64_t(tiles[ty].size());
}

void gather_rows_device(const double* W, int64_t ldw, const int32_t* d_rows, int64_t nrows, const int32_t* d_cols,
                        int64_t ncols, double* out, hipStream_t s) {
    for (int64_t r0 = 0; r0 < nrows; r0 += 65535) {
        const int64_t nr = std::min<int64_t>(65535, nrows - r0);
        hipLaunchKernelGGL(k_gather_rows, dim3(gblocks(ncols), unsigned(nr)), dim3(256), 0, s, W, ldw, d_rows + r0, d_cols, ncols,
                           out + r0 * ncols);
    }
    HIP_CHECK(hipGetLastError());
}

void permute_cols_device(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t N, int k, const int32_t* idx,
                         hipStream_t s) {
    if (N <= 0 || k <= 0) return;
    hipLaunchKernelGGL(k_permute_cols, dim3(gblocks(N), unsigned(k)), dim3(256), 0, s, src, lds, dst, ldd, N, idx);
    HIP_CHECK(hipGetLastError());
}

void matvec_device(const bem_problem* p, bool fp32, const double* d_x, int64_t ldx, int k, double* d_y, hipStream_t s,
                   const int* gate) {
    if (p->N == 0) return;
    double* part = p->mv_partial.as<double>();
    if (fp32) {
        if (!p->W32.ptr) fail(BEM_E_INVALID_ARG, "problem has no FP32 matrix (assemble with BEM_FP32_REFINE)");
        launch_matvec<float, double>(p, p->W32.as<float>(), d_x, ldx, k, d_y, ldx, s, static_cast<float*>(p->mv_xt.ptr),
                                     part, static_cast<float*>(p->mv_sym.ptr), gate);
    } else {
        launch_matvec<double, double>(p, p->W64.as<double>(), d_x, ldx, k, d_y, ldx, s, p->mv_xt.as<double>(), part,
                                      static_cast<double*>(p->mv_sym.ptr), gate);
    }
}

// ---- products that allocate nothing ------------------------------------------------------------
// bem_matvec_noalloc keeps the transposed right-hand sides and the partial sums of its product in
// this file-scope device array instead of the problem's buffers.  Each device holds its own copy,
// at its own address, until the process ends; host code uses only the address that
// hipGetSymbolAddress returns for the current device (the array's name is a host-side stand-in
// there, not a device address).  Calls on one device share it: overlapping calls race.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

void* noalloc_scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) fail(BEM_E_INVALID_ARG, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        HIP_CHECK(hipGetDevice(&cur));
        if (cur != device) HIP_CHECK(hipSetDevice(device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            fail(BEM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

// layout: the transposed right-hand sides, then either the block-row partials of the symmetric
// product or (a matrix of one 64-row block) the split partials of the plain one, then, for a
// renumbered problem, x and y of the product in the internal dof order (k x N each)
size_t noalloc_matvec_bytes(const bem_problem* p, bool fp32, int k) {
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    const size_t xt = align256(16 * size_t(p->ldw) * es);
    const int ty = fp32 ? 0 : 1;
    const size_t part = p->mv_ntiles[ty] > 0 ? size_t(p->ldw / 64) * size_t(p->mv_nst[ty] + 1) * 1024 * es
                                             : 16 * 16 * size_t(p->ldw) * sizeof(double);
    const size_t perm = p->renumbered ? 2 * align256(size_t(k) * size_t(p->N) * sizeof(double)) : 0;
    return xt + align256(part) + perm;
}

void matvec_device_noalloc(const bem_problem* p, bool fp32, const double* d_x, int64_t ldx, int k, double* d_y,
                           hipStream_t s, void* scr) {
    if (p->N == 0) return;
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    unsigned char* base = static_cast<unsigned char*>(scr);
    void* xt = base;
    void* sp = base + align256(16 * size_t(p->ldw) * es);     // one of the two partial layouts is used
    double* part = static_cast<double*>(sp);
    const double* x = d_x;
    double* y = d_y;
    int64_t ld = ldx;
    if (p->renumbered) {   // the product runs in the internal order, between two permutations
        const int ty = fp32 ? 0 : 1;
        const size_t partb = p->mv_ntiles[ty] > 0 ? size_t(p->ldw / 64) * size_t(p->mv_nst[ty] + 1) * 1024 * es
                                                  : 16 * 16 * size_t(p->ldw) * sizeof(double);
        double* xi = reinterpret_cast<double*>(base + align256(16 * size_t(p->ldw) * es) + align256(partb));
        double* yi = xi + align256(size_t(k) * size_t(p->N) * sizeof(double)) / sizeof(double);
        permute_cols_device(d_x, ldx, xi, p->N, p->N, k, p->d_dof_user.as<int32_t>(), s);
        x = xi;
        y = yi;
        ld = p->N;
    }
    if (fp32) {
        if (!p->W32.ptr) fail(BEM_E_INVALID_ARG, "problem has no FP32 matrix (assemble with BEM_FP32_REFINE)");
        launch_matvec<float, double>(p, p->W32.as<float>(), x, ld, k, y, ld, s, static_cast<float*>(xt), part,
                                     static_cast<float*>(sp), nullptr);
    } else {
        launch_matvec<double, double>(p, p->W64.as<double>(), x, ld, k, y, ld, s, static_cast<double*>(xt), part,
                                      static_cast<double*>(sp), nullptr);
    }
    if (p->renumbered) permute_cols_device(y, p->N, d_y, ldx, p->N, k, p->d_dof_int.as<int32_t>(), s);
}

// ---------------------------------------------------------------------------------------------
// PCG on device buffers.  b, x: [k][ld].  x is used as the start vector (zero it for x0 = 0) and
// receives the result.  Per-column tolerance tol[c] on ||r|| / ||b||.
// ---------------------------------------------------------------------------------------------
struct PcgResult {
    std::vector<int> iters, flag, active, refreshes;
    std::vector<double> rr, bb, cond;
    bool graphed = false;
};

// Block (P)CG on device buffers.  b, x: [k][ld]; x is the start vector (zero it for x0 = 0) and
// receives the result; per-column tolerance tol[c] on ||r|| / ||b||.
// mixed = false: FP64 matrix and factors; the recurrence residual decides convergence.
// mixed = true: products with the FP32 matrix and FP32 block inverses (FP64 vectors, dots and coarse
// solve), with reliable updates: the recurrence residual is replaced by the true residual
// b - W x with the FP64 matrix whenever it has fallen by `refresh` since the last replacement, and
// before any column is declared converged, so convergence is always judged on a true residual.  The
// device decides in each iteration which columns are due; the FP64 product of x is gated on any
// column being due, so one captured iteration serves every case and the host only polls.
// slots != nullptr (serving): b and x are the slot buffers (zero at the start, every column
// inactive), columns are started and collected through the hooks at the check points, and
// max_iter bounds each column's iterations instead of the launches.
PcgResult pcg_device(bem_problem* p, const bem_precond* M, bool mixed, const double* b, double* x, bool x_nonzero,
                     int k, int64_t ld, const std::vector<double>& tol, int max_iter, int check_every, bool use_graph,
                     bool want_cond, double refresh, PcgSlots* slots = nullptr) {
    hipStream_t s = p->stream;
    const int64_t N = p->N;
    const unsigned G = gblocks(N);
    const bool fp32 = mixed;
    DeviceBuffer r(sizeof(double) * ld * k, s), z(sizeof(double) * ld * k, s), pp(sizeof(double) * ld * k, s), q(sizeof(double) * ld * k, s);
    DeviceBuffer part(sizeof(double) * G * k * 3, s), dst(sizeof(ColState) * k, s), dtol(sizeof(double) * k, s);
    DeviceBuffer dgate(sizeof(int) * 2, s);   // any column active, any column due (k_gate)
    const int max_hist = want_cond ? std::max(1, max_iter) : 1;
    DeviceBuffer hist(sizeof(double) * 2 * max_hist * k, s);
    DeviceBuffer cscr(sizeof(double) * (M ? precond_scratch_size(M, std::min(k, 16)) : 1), s);
    std::vector<double> tol2(k);
    for (int c = 0; c < k; ++c) tol2[c] = tol[c] * tol[c];
    HIP_CHECK(hipMemcpyAsync(dtol.ptr, tol2.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    double* pa = part.as<double>();
    double* pb = pa + int64_t(G) * k;
    double* pc = pb + int64_t(G) * k;
    const dim3 vg(G, unsigned(k)), vb(256);

    auto apply_M = [&](const double* in, double* out) {
        if (M) precond_apply_device(M, fp32, in, ld, k, out, s, cscr.as<double>());
        else hipLaunchKernelGGL(k_copy, vg, vb, 0, s, in, out, ld, N);
        HIP_CHECK(hipGetLastError());
    };

    // ---- initial state ----
    if (x_nonzero) {
        matvec_device(p, false, x, ld, k, q.as<double>(), s);
        hipLaunchKernelGGL(k_residual, vg, vb, 0, s, b, q.as<double>(), r.as<double>(), ld, N);
    } else {
        hipLaunchKernelGGL(k_copy, vg, vb, 0, s, b, r.as<double>(), ld, N);
    }
    apply_M(r.as<double>(), z.as<double>());
    hipLaunchKernelGGL(k_copy, vg, vb, 0, s, z.as<double>(), pp.as<double>(), ld, N);
    hipLaunchKernelGGL(k_dot_partial, vg, vb, 0, s, b, b, ld, N, pa);
    hipLaunchKernelGGL(k_dot_partial, vg, vb, 0, s, r.as<double>(), r.as<double>(), ld, N, pb);
    hipLaunchKernelGGL(k_dot_partial, vg, vb, 0, s, r.as<double>(), z.as<double>(), ld, N, pc);
    hipLaunchKernelGGL(k_init_state, dim3(k), vb, 0, s, pa, pb, pc, int(G), dtol.as<double>(), dst.as<ColState>());
    HIP_CHECK(hipGetLastError());

    ColState* st = dst.as<ColState>();
    double* h = hist.as<double>();
    int* gate = dgate.as<int>();
    // one (P)CG iteration.  The product with p is skipped once no column is active; mixed: when a
    // column is due for replacement, every active column gets r = b - W x in FP64 after the update
    // of x (q is free by then and holds W x); that product runs only then.
    auto iteration = [&]() {
        hipLaunchKernelGGL(k_gate, dim3(1), vb, 0, s, st, k, 0, gate);
        matvec_device(p, fp32, pp.as<double>(), ld, k, q.as<double>(), s, gate);
        hipLaunchKernelGGL(k_dot_partial, vg, vb, 0, s, pp.as<double>(), q.as<double>(), ld, N, pa);
        hipLaunchKernelGGL(k_alpha, dim3(k), vb, 0, s, pa, int(G), st, h, max_hist);
        hipLaunchKernelGGL(k_update_xr, vg, vb, 0, s, x, r.as<double>(), pp.as<double>(), q.as<double>(), ld, N, st, pb);
        if (mixed) {
            hipLaunchKernelGGL(k_check_due, dim3(k), vb, 0, s, pb, int(G), st, refresh * refresh);
            hipLaunchKernelGGL(k_gate, dim3(1), vb, 0, s, st, k, 1, gate);
            matvec_device(p, false, x, ld, k, q.as<double>(), s, gate + 1);
            hipLaunchKernelGGL(k_residual_due, vg, vb, 0, s, b, q.as<double>(), r.as<double>(), ld, N, st, pb, gate);
        }
        hipLaunchKernelGGL(k_check, dim3(k), vb, 0, s, pb, int(G), st, mixed ? 1 : 0, gate);
        apply_M(r.as<double>(), z.as<double>());
        hipLaunchKernelGGL(k_dot_partial, vg, vb, 0, s, r.as<double>(), z.as<double>(), ld, N, pc);
        hipLaunchKernelGGL(k_beta, dim3(k), vb, 0, s, pc, int(G), st, h, max_hist);
        hipLaunchKernelGGL(k_update_p, vg, vb, 0, s, pp.as<double>(), z.as<double>(), ld, N, st);
    };

    // the captured iteration; an exception between begin and end of a capture still ends it, so
    // the stream never stays in capture mode.  The graph is destroyed under the capture mutex, like
    // every other call that may wait on the device: destroying an executable graph can wait for its
    // launches, which must not happen while another thread's capture is open.
    struct Graph {
        hipStream_t s;
        bool capturing = false;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        ~Graph() {
            std::lock_guard<std::mutex> lk(capture_mutex());
            if (capturing) {
                hipGraph_t g = nullptr;
                if (hipStreamEndCapture(s, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
            }
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
        }
    } gr{s};
    // A capture that fails with a capture error (the runtime ends a capture when a call elsewhere
    // in the process is not permitted alongside it) queued no work: the solve then launches its
    // iterations directly, with the same kernels and results.
    auto capture_error = [](hipError_t e) {
        return e == hipErrorStreamCaptureUnsupported || e == hipErrorStreamCaptureInvalidated ||
               e == hipErrorStreamCaptureMerge || e == hipErrorStreamCaptureUnmatched ||
               e == hipErrorStreamCaptureUnjoined || e == hipErrorStreamCaptureIsolation ||
               e == hipErrorStreamCaptureImplicit || e == hipErrorCapturedEvent ||
               e == hipErrorStreamCaptureWrongThread;
    };
    bool graphed = false;
    if (use_graph) {
        std::lock_guard<std::mutex> lk(capture_mutex());   // no device-wide synchronisation meanwhile
        graphed = true;
        {
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                gr.capturing = true;
                try {
                    iteration();
                    e = hipGetLastError();
                } catch (const Failure&) {
                    // a launch inside the capture reported an error (the runtime invalidates a
                    // capture when a call elsewhere in the process is not permitted beside it):
                    // the capture is dropped and the direct launches below redo the same work, or
                    // report the error if it is not the capture's
                    e = hipGetLastError();
                    if (e == hipSuccess) e = hipErrorStreamCaptureInvalidated;
                }
                hipGraph_t g = nullptr;
                const hipError_t e_end = hipStreamEndCapture(s, &g);
                gr.capturing = false;
                gr.graph = g;
                if (e == hipSuccess) e = e_end;
                if (e == hipSuccess && !g) e = hipErrorStreamCaptureInvalidated;
            }
            if (e == hipSuccess) {
                HIP_CHECK(hipGraphInstantiate(&gr.exec, gr.graph, nullptr, nullptr, 0));
            } else if (capture_error(e)) {
                (void)hipGetLastError();
                graphed = false;
                // an invalidated capture can leave the stream in capture mode: end it again, and
                // refuse to go on with a stream that stays there
                hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
                for (int tries = 0; tries < 2; ++tries) {
                    if (hipStreamIsCapturing(s, &cs) != hipSuccess) cs = hipStreamCaptureStatusInvalidated;
                    if (cs == hipStreamCaptureStatusNone) break;
                    hipGraph_t g2 = nullptr;
                    if (hipStreamEndCapture(s, &g2) == hipSuccess && g2) (void)hipGraphDestroy(g2);
                    (void)hipGetLastError();
                }
                if (cs != hipStreamCaptureStatusNone)
                    fail(BEM_E_DEVICE, "the problem's stream stayed in capture mode after an invalidated capture");
            } else {
                HIP_CHECK(e);
            }
        }
    }
    auto launch = [&]() {
        if (graphed) {
            HIP_CHECK(hipGraphLaunch(gr.exec, s));
        } else {
            iteration();
            HIP_CHECK(hipGetLastError());
        }
    };
    std::vector<ColState> hs(k);
    int launched = 0;
    const int every = std::max(1, check_every);
    HIP_CHECK(hipMemcpyAsync(hs.data(), st, sizeof(ColState) * k, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    auto any_active = [&]() {
        for (auto& c : hs) if (c.active) return true;
        return false;
    };

    // serving: collect the stopped columns, stop the ones out of iterations, start new ones
    std::vector<char> owned(size_t(k), 0);
    std::vector<double> hg(3 * static_cast<size_t>(k)), htol2(static_cast<size_t>(k));
    DeviceBuffer dg(slots ? sizeof(double) * 3 * k : 8, s);
    auto serve_check = [&]() -> bool {
        bool changed = false;
        for (int c = 0; c < k; ++c)
            if (owned[c] && hs[c].active && hs[c].iters >= max_iter) {
                hipLaunchKernelGGL(k_stop_column, dim3(1), dim3(1), 0, s, st + c);
                hs[c].active = 0;
                changed = true;
            }
        if (changed) HIP_CHECK(hipStreamSynchronize(s));
        std::vector<int> free_slots;
        int running = 0;
        for (int c = 0; c < k; ++c) {
            if (owned[c] && !hs[c].active) {
                PcgColumnResult cr;
                cr.iters = hs[c].iters;
                cr.refreshes = hs[c].refreshes;
                cr.relres = hs[c].bb > 0 ? std::sqrt(hs[c].rr / hs[c].bb) : 0.0;
                cr.status = hs[c].flag ? BEM_E_BREAKDOWN : (hs[c].rr <= hs[c].tol2 * hs[c].bb ? BEM_OK : BEM_E_NOT_CONVERGED);
                slots->finished(c, x + int64_t(c) * ld, cr);
                owned[c] = 0;
            }
            if (!owned[c]) free_slots.push_back(c);
            else ++running;
        }
        std::vector<PcgNewColumn> start;
        slots->admit(free_slots, running, start);
        if (start.empty()) return running > 0;
        const dim3 g1(G, 1);
        for (const PcgNewColumn& nc : start) {
            const int c = nc.slot;
            if (c < 0 || c >= k || owned[c]) fail(BEM_E_INVALID_ARG, "serving: column slot not free");
            std::copy(nc.g, nc.g + 3, &hg[size_t(3) * c]);
            htol2[c] = nc.tol * nc.tol;
            HIP_CHECK(hipMemcpyAsync(dg.as<double>() + 3 * c, &hg[size_t(3) * c], sizeof(double) * 3, hipMemcpyHostToDevice, s));
            HIP_CHECK(hipMemcpyAsync(dtol.as<double>() + c, &htol2[c], sizeof(double), hipMemcpyHostToDevice, s));
            double* bc = const_cast<double*>(b) + int64_t(c) * ld;
            rhs_device(p, dg.as<double>() + 3 * c, 1, bc, s);
            hipLaunchKernelGGL(k_fill, dim3(G), vb, 0, s, x + int64_t(c) * ld, 0.0, N);
            hipLaunchKernelGGL(k_copy, g1, vb, 0, s, bc, r.as<double>() + int64_t(c) * ld, ld, N);
        }
        apply_M(r.as<double>(), z.as<double>());   // every slot: z is scratch between iterations
        for (const PcgNewColumn& nc : start) {
            const int c = nc.slot;
            const int64_t o = int64_t(c) * ld;
            const double* bc = b + o;
            hipLaunchKernelGGL(k_copy, g1, vb, 0, s, z.as<double>() + o, pp.as<double>() + o, ld, N);
            hipLaunchKernelGGL(k_dot_partial, g1, vb, 0, s, bc, bc, ld, N, pa + int64_t(c) * G);
            hipLaunchKernelGGL(k_dot_partial, g1, vb, 0, s, r.as<double>() + o, r.as<double>() + o, ld, N, pb + int64_t(c) * G);
            hipLaunchKernelGGL(k_dot_partial, g1, vb, 0, s, r.as<double>() + o, z.as<double>() + o, ld, N, pc + int64_t(c) * G);
            hipLaunchKernelGGL(k_init_state, dim3(1), vb, 0, s, pa + int64_t(c) * G, pb + int64_t(c) * G, pc + int64_t(c) * G,
                               int(G), dtol.as<double>() + c, st + c);
            owned[c] = 1;
        }
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(hs.data(), st, sizeof(ColState) * k, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        return true;
    };
    if (slots) slots->graphed = graphed;
    for (;;) {
        if (slots) {
            // the hooks decide when the batch ends; columns that stop on their start (zero
            // right-hand side) are reported at the next check without an iteration
            if (!any_active()) {
                if (!serve_check()) break;
                if (!any_active()) continue;
            }
        } else if (!(any_active() && launched < max_iter)) {
            break;
        }
        // (serving: max_iter bounds each column, through serve_check, not the launches)
        const int n = slots ? every : std::min(every, max_iter - launched);
        for (int i = 0; i < n; ++i) launch();
        launched += n;
        HIP_CHECK(hipMemcpyAsync(hs.data(), st, sizeof(ColState) * k, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (slots && !serve_check()) break;
    }
    PcgResult res;
    res.graphed = graphed;
    res.iters.resize(k); res.flag.resize(k); res.active.resize(k); res.rr.resize(k); res.bb.resize(k); res.cond.assign(k, std::nan(""));
    res.refreshes.resize(k);
    std::vector<double> hh;
    if (want_cond) {
        hh.resize(size_t(2) * max_hist * k);
        HIP_CHECK(hipMemcpyAsync(hh.data(), h, sizeof(double) * hh.size(), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
    }
    for (int c = 0; c < k; ++c) {
        res.iters[c] = hs[c].iters;
        res.flag[c] = hs[c].flag;
        res.active[c] = hs[c].active;
        res.rr[c] = hs[c].rr;
        res.bb[c] = hs[c].bb;
        res.refreshes[c] = hs[c].refreshes;
        if (want_cond && hs[c].iters > 0 && !hs[c].flag) {
            const int m = std::min(hs[c].iters, max_hist);
            res.cond[c] = lanczos_condition(&hh[size_t(c) * 2 * max_hist], &hh[size_t(c) * 2 * max_hist + max_hist], m);
        }
    }
    return res;
}

// ---------------------------------------------------------------------------------------------
// Full solve: FP64 PCG, or FP32-matrix PCG corrections inside FP64 iterative refinement.
// b: device [k][N]; x: device [k][N] (output).
// ---------------------------------------------------------------------------------------------
void solve_device(bem_problem* p, const bem_precond* M, const double* b, double* x, int k, const bem_solve_opts& o,
                  bem_solve_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = p->stream;
    const int64_t N = p->N, ld = N;
    const unsigned G = gblocks(N);
    const dim3 vg(G, unsigned(k)), vb(256);
    const bool use_m = (M != nullptr) && o.use_precond;
    const int check = o.check_every > 0 ? o.check_every : 4;
    std::vector<int> iters(k, 0), outer(k, 0), status(k, BEM_OK);
    std::vector<double> relres(k, 0.0), cond(k, std::nan(""));

    const bool x_nonzero = o.x0 != nullptr;
    if (x_nonzero) HIP_CHECK(hipMemcpyAsync(x, o.x0, sizeof(double) * ld * k, hipMemcpyHostToDevice, s));
    else hipLaunchKernelGGL(k_fill, dim3(256), vb, 0, s, x, 0.0, int64_t(k) * ld);
    bool final_check = true, graphed = false;
    if (o.precision == BEM_FP64) {
        std::vector<double> tol(k, o.tol);
        PcgResult r = pcg_device(p, use_m ? M : nullptr, false, b, x, x_nonzero, k, ld, tol, o.max_iter, check, o.use_graph != 0, true,
                                 0.0);
        graphed = r.graphed;
        for (int c = 0; c < k; ++c) {
            iters[c] = r.iters[c];
            cond[c] = r.cond[c];
            if (r.flag[c]) status[c] = BEM_E_BREAKDOWN;
            else if (r.active[c]) status[c] = BEM_E_NOT_CONVERGED;
        }
    } else {
        if (!p->W32.ptr) fail(BEM_E_INVALID_ARG, "mixed precision needs a problem assembled with BEM_FP32_REFINE");
        if (use_m && !M->inv32.ptr) fail(BEM_E_INVALID_ARG, "mixed precision needs a preconditioner with factor_fp32 = 1");
        std::vector<double> tol(k, o.tol);
        const double refresh = (o.refresh_factor > 0 && o.refresh_factor < 1) ? o.refresh_factor : kRefreshDefault;
        PcgResult r = pcg_device(p, use_m ? M : nullptr, true, b, x, x_nonzero, k, ld, tol, o.max_iter, check, o.use_graph != 0, true,
                                 refresh);
        graphed = r.graphed;
        final_check = false;
        for (int c = 0; c < k; ++c) {
            iters[c] = r.iters[c];
            outer[c] = r.refreshes[c];
            cond[c] = r.cond[c];
            // a converged column stopped on a true FP64 residual: its relres is already exact
            relres[c] = r.bb[c] > 0 ? std::sqrt(r.rr[c] / r.bb[c]) : 0.0;
            if (r.flag[c]) status[c] = BEM_E_BREAKDOWN;
            else if (r.active[c]) status[c] = BEM_E_NOT_CONVERGED;
            if (status[c] != BEM_OK) final_check = true;
        }
    }
    // true FP64 residual of the result
    if (final_check) {
        DeviceBuffer y(sizeof(double) * ld * k, s), r(sizeof(double) * ld * k, s), part(sizeof(double) * G * k * 2, s);
        matvec_device(p, false, x, ld, k, y.as<double>(), s);
        hipLaunchKernelGGL(k_residual, vg, vb, 0, s, b, y.as<double>(), r.as<double>(), ld, N);
        hipLaunchKernelGGL(k_dot_partial, vg, vb, 0, s, r.as<double>(), r.as<double>(), ld, N, part.as<double>());
        hipLaunchKernelGGL(k_dot_partial, vg, vb, 0, s, b, b, ld, N, part.as<double>() + int64_t(G) * k);
        std::vector<double> hp(size_t(2) * G * k);
        HIP_CHECK(hipMemcpyAsync(hp.data(), part.ptr, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        for (int c = 0; c < k; ++c) {
            double a = 0, bsum = 0;
            for (unsigned g = 0; g < G; ++g) { a += hp[size_t(c) * G + g]; bsum += hp[size_t(G) * k + size_t(c) * G + g]; }
            relres[c] = bsum > 0 ? std::sqrt(a / bsum) : 0.0;
        }
    }
    const double tt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int c = 0; c < k; ++c) {
            info[c].iters = iters[c];
            info[c].outer_iters = outer[c];
            info[c].status = status[c];
            info[c].graph = graphed ? 1 : 0;
            info[c].relres = relres[c];
            info[c].est_cond = cond[c];
            info[c].t_total_s = tt;
        }
}

void pcg_serve(bem_problem* p, const bem_precond* M, bool mixed, int slots, int max_iter, int check_every,
               PcgSlots& hooks) {
    if (slots < 1) fail(BEM_E_INVALID_ARG, "serving: no column slots");
    if (mixed && !p->W32.ptr) fail(BEM_E_INVALID_ARG, "mixed precision needs a problem assembled with BEM_FP32_REFINE");
    if (mixed && M && !M->inv32.ptr) fail(BEM_E_INVALID_ARG, "mixed precision needs a preconditioner with factor_fp32 = 1");
    hipStream_t s = p->stream;
    const int64_t ld = p->N;
    DeviceBuffer b(sizeof(double) * std::max<int64_t>(1, ld * slots), s), x(sizeof(double) * std::max<int64_t>(1, ld * slots), s);
    hipLaunchKernelGGL(k_fill, dim3(256), dim3(256), 0, s, b.as<double>(), 0.0, ld * slots);
    hipLaunchKernelGGL(k_fill, dim3(256), dim3(256), 0, s, x.as<double>(), 0.0, ld * slots);
    HIP_CHECK(hipGetLastError());
    std::vector<double> tol(size_t(slots), 1.0);   // every slot starts inactive (b = 0)
    pcg_device(p, M, mixed, b.as<double>(), x.as<double>(), false, slots, ld, tol, max_iter, check_every, true, false, kRefreshDefault,
               &hooks);
}

}  // namespace bem
