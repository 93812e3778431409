// Two-level substructuring additive Schwarz preconditioner (paper: eq. jumpSplit in Section 6.4,
// the Remark on duplicate face copies after it, and the Remark "Bound on the number of
// Preconditioned Conjugate Gradient iterations"):
//
//   M r = sum_F R_F^T W_FF^{-1} R_F r + R_W^T W_WW^{-1} R_W r + R_H^T (R_H W R_H^T)^{-1} R_H r.
//
// The face and wire-basket spaces are spanned by fine jump basis functions (the discrete harmonic
// extensions omega_{i,j} keep the traces of phi_{i,j}, Lemma lemdof), so R_F, R_W are 0/1 dof
// restrictions and their blocks are principal submatrices of W.  Face dofs of a patch: dofs at
// vertices whose triangles all lie in that patch and with q = 2; the rest is the wire basket.
// The coarse space is the jump space of a nested coarse mesh written in the fine basis.
//
// Device work: every block (faces, wire basket, coarse Galerkin matrix) is gathered into a padded
// 64-multiple square and inverted explicitly by symmetric block Gauss-Jordan elimination on 64x64
// tiles (FP64 matrix cores for the trailing updates).  All blocks of uneven sizes advance together:
// each launch carries one tile step of every block that still has work (ragged batching).
// Applying M is then a ragged batch of dense row-panel products.  With the diagonal wire basket
// (Remark "Approximate solvers") that block is replaced by 1 / W_dd on its dofs.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <numeric>
#include <tuple>

#include "internal.h"
#include "strips.h"

namespace bem {

namespace {

constexpr int TBK = 64;     // tile edge
constexpr int LDT = 65;     // LDS leading dimension (padding against bank conflicts)

struct BlockMeta { int64_t n, npad, idx_off, mat_off, xoff; };

// Tile moves by a block of 256 threads (every launch of the kernels below uses 256): thread t moves
// elements t + 256 q, q < 16.  All 16 loads of a thread are issued before the first is used, so a
// tile costs one memory latency instead of sixteen.
constexpr int kTilePer = TBK * TBK / 256;

__device__ __forceinline__ void tile_store(const double* __restrict__ s, double* __restrict__ g, int64_t ld) {
    double v[kTilePer];
#pragma unroll
    for (int q = 0; q < kTilePer; ++q) {
        const int e = threadIdx.x + 256 * q;
        v[q] = s[(e >> 6) * LDT + (e & 63)];
    }
#pragma unroll
    for (int q = 0; q < kTilePer; ++q) {
        const int e = threadIdx.x + 256 * q;
        g[int64_t(e >> 6) * ld + (e & 63)] = v[q];
    }
}

// LDS tile <- sign * G^T (G a 64 x 64 tile in global memory with row stride ld)
__device__ __forceinline__ void tile_load_t(double* __restrict__ s, const double* __restrict__ g, int64_t ld, double sign) {
    double v[kTilePer];
#pragma unroll
    for (int q = 0; q < kTilePer; ++q) {
        const int e = threadIdx.x + 256 * q;
        v[q] = g[int64_t(e >> 6) * ld + (e & 63)];
    }
#pragma unroll
    for (int q = 0; q < kTilePer; ++q) {
        const int e = threadIdx.x + 256 * q;
        s[(e & 63) * LDT + (e >> 6)] = sign * v[q];
    }
}

// --- gather: A_b = W[idx_b, idx_b] padded with the identity ---------------------------------
__global__ __launch_bounds__(256) void k_gather(const int4* __restrict__ tasks, const BlockMeta* __restrict__ meta,
                                                const int32_t* __restrict__ idx, const double* __restrict__ W,
                                                int64_t ldw, double shift, double* __restrict__ A) {
    const int4 t = tasks[blockIdx.x];
    const BlockMeta m = meta[t.x];
    const int32_t* id = idx + m.idx_off;
    double* a = A + m.mat_off;
    double v[kTilePer];   // all of a thread's loads in flight before the stores
#pragma unroll
    for (int q = 0; q < kTilePer; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int64_t r = int64_t(t.y) * TBK + (e >> 6), c = int64_t(t.z) * TBK + (e & 63);
        v[q] = (r < m.n && c < m.n) ? W[int64_t(id[r]) * ldw + id[c]] + ((r == c) ? shift : 0.0) : ((r == c) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < kTilePer; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int64_t r = int64_t(t.y) * TBK + (e >> 6), c = int64_t(t.z) * TBK + (e & 63);
        a[r * m.npad + c] = v[q];
    }
}

// --- block Gauss-Jordan inversion, 128-wide pivots ----------------------------------------------
// Each block B (a face, the wire basket, the coarse Galerkin matrix; SPD, padded with the identity
// to a multiple of 128) is overwritten by its inverse.  Step k eliminates the k-th 128-wide block
// row and column.  With P = (S_kk)^{-1} of the current state S:  S_kj <- P S_kj (row k),
// S_ik <- -S_ik P (column k),  S_ij <- S_ij - S_ik P S_kj (i, j != k),  S_kk <- P.  Pivot blocks
// of an SPD matrix stay SPD, so no pivoting is needed.  The state keeps a signed symmetry:
// S_ij = s S_ji^T with s = -1 exactly when one of i, j has been eliminated, so only the lower tiles
// (i >= j) are stored and updated; an upper tile is read as the signed transpose of its mirror.
// At the end every index is eliminated and the lower tiles hold the (symmetric) inverse, which
// is then mirrored into the upper tiles.  The whole lower triangle is read and written once per
// step, so 128-wide pivots halve the passes over the matrix against 64-wide ones, and every tile
// update is a 128 x 128 x 128 product on the FP64 matrix cores.
// A step is three launches.  k_gj_row stages, for every j != k, the old column value C_j = S_jk,
// the new row value R_j = P S_kj and, for j > k, the new column tile D_j = -S_jk P.  k_gj_update
// applies S_ij -= C_i R_j to the lower tiles off row and column k and copies the new row / column
// / pivot tiles in (the next pivot's tile first).  k_gj_pivot inverts the updated tile (k+1, k+1):
// the pivot inverse of step k+1.  No launch writes a tile that it also reads.
constexpr int TB2 = 128;   // pivot width and tile edge
constexpr int KC2 = 16;    // K chunk of the tile products
constexpr int LS2 = 144;   // LDS row stride (doubles) of a staged chunk: lanes 0-31 and 32-63 of a read
                           // hit disjoint banks (2 x 144 = 32 mod 64 banks between consecutive k)
constexpr int NT2 = 512;   // threads of every elimination launch: 8 waves

// A 128 x 128 operand M in global memory: M(r, c) = sign * (stored transposed ? p[c ld + r] : p[r ld + c]).
// A K-chunk of an A operand is staged as st[k][x] = A(x, k0 + k), of a B operand as st[k][x] = B(k0 + k, x);
// xcontig tells whether x runs along the stored rows (coalesced either way).
struct Opnd {
    const double* p;
    int64_t ld;
    bool xcontig;
    double sign;
};
__device__ __forceinline__ Opnd opnd_a(const double* p, int64_t ld, bool trans, double sign) { return Opnd{p, ld, trans, sign}; }
__device__ __forceinline__ Opnd opnd_b(const double* p, int64_t ld, bool trans, double sign) { return Opnd{p, ld, !trans, sign}; }

// thread t fetches 4 consecutive stored doubles of the chunk at k0
__device__ __forceinline__ void chunk_fetch(double (&v)[4], const Opnd& o, int k0) {
    const int t = threadIdx.x;
    const double* q = o.xcontig ? o.p + int64_t(k0 + (t >> 5)) * o.ld + (t & 31) * 4
                                : o.p + int64_t(t >> 2) * o.ld + k0 + (t & 3) * 4;
    const double2 d0 = *reinterpret_cast<const double2*>(q), d1 = *reinterpret_cast<const double2*>(q + 2);
    v[0] = d0.x;
    v[1] = d0.y;
    v[2] = d1.x;
    v[3] = d1.y;
}

__device__ __forceinline__ void chunk_put(double* __restrict__ st, const double (&v)[4], const Opnd& o) {
    const int t = threadIdx.x;
    if (o.xcontig) {
        double* d = st + (t >> 5) * LS2 + (t & 31) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = o.sign * v[j];
    } else {
        const int x = t >> 2, kb = (t & 3) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) st[(kb + j) * LS2 + x] = o.sign * v[j];
    }
}

// acc += A B, A and B 128 x 128 operands, on the FP64 matrix cores.  Wave w = 4 wr + wc computes
// rows 64 wr .. 64 wr + 63 x columns 32 wc .. 32 wc + 31 as 4 x 2 tiles of 16 x 16; lane l = 16 kk + i
// supplies A[row i][k kk] and B[k kk][column i] to each 16x16x4 step, and register r of
// acc[mt][nt] holds C[64 wr + 16 mt + kk + 4 r][32 wc + 16 nt + i].  K runs in chunks of 16 through
// two LDS buffers per operand (sa, sb: 2 x KC2 x LS2 each): chunk c is used from buffer c % 2 while
// chunk c + 1 is staged into the other one and chunk c + 2 is loaded into registers, one barrier
// per chunk.
__device__ __forceinline__ void gemm128(f64x4 (&acc)[4][2], const Opnd& A, const Opnd& B, double* __restrict__ sa,
                                        double* __restrict__ sb) {
    constexpr int NCH = TB2 / KC2;
    constexpr int BUF = KC2 * LS2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kk = lane >> 4;
    const int wr = w >> 2, wc = w & 3;
    double va[4], vb[4];
    chunk_fetch(va, A, 0);
    chunk_fetch(vb, B, 0);
    __syncthreads();   // earlier readers of the buffers are done
    chunk_put(sa, va, A);
    chunk_put(sb, vb, B);
    chunk_fetch(va, A, KC2);
    chunk_fetch(vb, B, KC2);
    __syncthreads();
    for (int c = 0; c < NCH; ++c) {
        const double* ca = sa + (c & 1) * BUF;
        const double* cb = sb + (c & 1) * BUF;
#pragma unroll
        for (int ks = 0; ks < KC2 / 4; ++ks) {
            const int k = 4 * ks + kk;
            double a[4], b[2];
#pragma unroll
            for (int m = 0; m < 4; ++m) a[m] = ca[k * LS2 + 64 * wr + 16 * m + i];
#pragma unroll
            for (int n = 0; n < 2; ++n) b[n] = cb[k * LS2 + 32 * wc + 16 * n + i];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n) acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[n], acc[m][n], 0, 0, 0);
        }
        if (c + 1 < NCH) {
            // the other buffer was last read in chunk c - 1, before the previous barrier
            chunk_put(sa + ((c + 1) & 1) * BUF, va, A);
            chunk_put(sb + ((c + 1) & 1) * BUF, vb, B);
            __syncthreads();
            if (c + 2 < NCH) {
                chunk_fetch(va, A, (c + 2) * KC2);
                chunk_fetch(vb, B, (c + 2) * KC2);
            }
        }
    }
}

__device__ __forceinline__ void acc_zero(f64x4 (&acc)[4][2]) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = f64x4{0.0, 0.0, 0.0, 0.0};
}

// g (128 x 128, row stride ld) = scale * acc, or += scale * acc; each half of a thread's old values is
// read together before it is written
__device__ __forceinline__ void acc_store(const f64x4 (&acc)[4][2], double* __restrict__ g, int64_t ld, double scale,
                                          bool accumulate) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kk = lane >> 4;
    const int wr = w >> 2, wc = w & 3;
    double* g0 = g + int64_t(64 * wr + kk) * ld + 32 * wc + i;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double old[2][2][4];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    old[m][n][r] = accumulate ? g0[int64_t(16 * (2 * h + m) + 4 * r) * ld + 16 * n] : 0.0;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    g0[int64_t(16 * (2 * h + m) + 4 * r) * ld + 16 * n] = accumulate ? fma(scale, acc[2 * h + m][n][r], old[m][n][r])
                                                                                     : scale * acc[2 * h + m][n][r];
    }
}

// dst (128 x 128, row stride ldd) = M, M given as a B operand: each chunk stages rows k0 .. k0 + 15 of
// M, st[k][x] = M(k0 + k, x) (coalesced reads and writes also for a transposed source)
__device__ __forceinline__ void copy128(double* __restrict__ dst, int64_t ldd, const Opnd& M, double* __restrict__ st) {
    const int t = threadIdx.x;
    for (int c = 0; c < TB2 / KC2; ++c) {
        double v[4];
        chunk_fetch(v, M, c * KC2);
        __syncthreads();
        chunk_put(st, v, M);
        __syncthreads();
        const int r = t >> 5, x0 = (t & 31) * 4;
        *reinterpret_cast<double2*>(dst + int64_t(c * KC2 + r) * ldd + x0) = make_double2(st[r * LS2 + x0], st[r * LS2 + x0 + 1]);
        *reinterpret_cast<double2*>(dst + int64_t(c * KC2 + r) * ldd + x0 + 2) =
            make_double2(st[r * LS2 + x0 + 2], st[r * LS2 + x0 + 3]);
    }
}

// One elimination step kk = 8 q + RR of the 128 x 128 scalar Gauss-Jordan below, on this thread's
// 4 x 8 registers (rows 4 tr .., columns 8 tc ..): the owners of row and column kk publish them
// through LDS, then every element takes its new value without branches.
template <int RR>
__device__ __forceinline__ void gj128_step(double (&a)[32], int q, int tr, int tc, double* __restrict__ rowbuf,
                                           double* __restrict__ colbuf, bool& ok) {
    constexpr int RS = RR & 3;   // local row of kk in its owner
    const int kk = 8 * q + RR;
    double* rb = rowbuf + (RR & 1) * TB2;
    double* cb = colbuf + (RR & 1) * TB2;
    if (tr == 2 * q + (RR >> 2)) {
#pragma unroll
        for (int c = 0; c < 8; ++c) rb[8 * tc + c] = a[RS * 8 + c];
    }
    if (tc == q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) cb[4 * tr + r] = a[r * 8 + RR];
    }
    __syncthreads();
    const double piv = rb[kk];
    ok = ok && (piv > 0.0) && isfinite(piv);
    const double pinv = 1.0 / piv;
    double akj[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) akj[c] = rb[8 * tc + c];
    const bool colq = tc == q;   // this thread holds column kk (its local column RR)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const bool rowk = (4 * tr + r) == kk;
        const double aik = cb[4 * tr + r] * pinv;
        const double m = rowk ? 0.0 : aik;
        const double s = rowk ? pinv : 1.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            // row kk: akj * pinv; other rows: a - aik akj
            double v = rowk ? akj[c] * s : fma(-m, akj[c], a[r * 8 + c]);
            if (c == RR) v = colq ? (rowk ? pinv : -aik) : v;
            a[r * 8 + c] = v;
        }
    }
}

// In-place inverse of a 128 x 128 SPD matrix by scalar Gauss-Jordan without pivoting: src (row
// stride lds) -> dst (row stride ldd).  Thread (tr, tc) = (t >> 4, t & 15) of the 512 keeps rows
// 4 tr .. 4 tr + 3 x columns 8 tc .. 8 tc + 7 in registers; each step publishes the pivot row and
// column through LDS (alternating buffers, one barrier per step).  Returns false if a pivot was not
// positive and finite (then the matrix is not SPD).
__device__ __forceinline__ bool inverse128(const double* __restrict__ src, int64_t lds, double* __restrict__ dst, int64_t ldd,
                                           double* __restrict__ rowbuf, double* __restrict__ colbuf) {
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    double a[32];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 8; c += 2) {
            const double2 d = *reinterpret_cast<const double2*>(src + int64_t(4 * tr + r) * lds + 8 * tc + c);
            a[r * 8 + c] = d.x;
            a[r * 8 + c + 1] = d.y;
        }
    bool ok = true;
    for (int q = 0; q < TB2 / 8; ++q) {
        gj128_step<0>(a, q, tr, tc, rowbuf, colbuf, ok);
        gj128_step<1>(a, q, tr, tc, rowbuf, colbuf, ok);
        gj128_step<2>(a, q, tr, tc, rowbuf, colbuf, ok);
        gj128_step<3>(a, q, tr, tc, rowbuf, colbuf, ok);
        gj128_step<4>(a, q, tr, tc, rowbuf, colbuf, ok);
        gj128_step<5>(a, q, tr, tc, rowbuf, colbuf, ok);
        gj128_step<6>(a, q, tr, tc, rowbuf, colbuf, ok);
        gj128_step<7>(a, q, tr, tc, rowbuf, colbuf, ok);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 8; c += 2)
            *reinterpret_cast<double2*>(dst + int64_t(4 * tr + r) * ldd + 8 * tc + c) = make_double2(a[r * 8 + c], a[r * 8 + c + 1]);
    return ok;
}

// tile (row i, column j) of block m (64-wide tiles), row stride npad
__device__ __forceinline__ double* tile_at(double* a0, const BlockMeta& m, int i, int j) {
    return a0 + int64_t(i) * TBK * m.npad + int64_t(j) * TBK;
}

// tile (row i, column j) of block m (128-wide tiles), row stride npad
__device__ __forceinline__ double* tile2_at(double* a0, const BlockMeta& m, int i, int j) {
    return a0 + int64_t(i) * TB2 * m.npad + int64_t(j) * TB2;
}

// scratch of block b: C_j (old column values), R_j (new row values), D_j (new column tiles), at
// 3 npad x 128 per block, then two pivot tiles per block
__device__ __forceinline__ double* gj_C(double* scr, const BlockMeta& m, int j) { return scr + 3 * m.xoff * TB2 + int64_t(j) * TB2 * TB2; }
__device__ __forceinline__ double* gj_R(double* scr, const BlockMeta& m, int j) { return scr + (3 * m.xoff + m.npad) * TB2 + int64_t(j) * TB2 * TB2; }
__device__ __forceinline__ double* gj_D(double* scr, const BlockMeta& m, int j) { return scr + (3 * m.xoff + 2 * m.npad) * TB2 + int64_t(j) * TB2 * TB2; }

// the pivot inverse of step k lives in slot k % 2 of the block's two pivot tiles (the update
// launch of step k reads slot k % 2 while it writes slot (k+1) % 2)
__device__ __forceinline__ double* gj_piv(double* scr, int64_t pivot_off, int b, int k) {
    return scr + pivot_off + (int64_t(b) * 2 + (k & 1)) * TB2 * TB2;
}

// the first pivot inverse of every block (task (b, 0, 0))
__global__ __launch_bounds__(NT2) void k_gj_pivot0(const int4* __restrict__ tasks, const BlockMeta* __restrict__ meta,
                                                   double* __restrict__ A, double* __restrict__ scr, int64_t pivot_off,
                                                   int* __restrict__ flags) {
    __shared__ double rowbuf[2 * TB2], colbuf[2 * TB2];
    const int4 t = tasks[blockIdx.x];
    const BlockMeta m = meta[t.x];
    const bool ok = inverse128(tile2_at(A + m.mat_off, m, 0, 0), m.npad, gj_piv(scr, pivot_off, t.x, 0), TB2, rowbuf, colbuf);
    if (!ok && threadIdx.x == 0) flags[t.x] = 1;
}

// step k, task (b, k, j), j != k: the staging for column j
__global__ __launch_bounds__(NT2) void k_gj_row(const int4* __restrict__ tasks, const BlockMeta* __restrict__ meta,
                                                double* __restrict__ A, double* __restrict__ scr, int64_t pivot_off, int k) {
    __shared__ double sa[2 * KC2 * LS2], sb[2 * KC2 * LS2];
    const int4 t = tasks[blockIdx.x];
    const BlockMeta m = meta[t.x];
    const int j = t.z;
    double* a0 = A + m.mat_off;
    const double* piv = gj_piv(scr, pivot_off, t.x, k);
    // S_kj and S_jk from the stored lower tile of the pair
    const Opnd Pa = opnd_a(piv, TB2, false, 1.0), Pb = opnd_b(piv, TB2, false, 1.0);
    const Opnd Skj = j < k ? opnd_b(tile2_at(a0, m, k, j), m.npad, false, 1.0)    // stored
                           : opnd_b(tile2_at(a0, m, j, k), m.npad, true, 1.0);    // S_jk^T, both uneliminated
    f64x4 acc[4][2];
    acc_zero(acc);
    gemm128(acc, Pa, Skj, sa, sb);                                               // R_j = P S_kj
    acc_store(acc, gj_R(scr, m, j), TB2, 1.0, false);
    // C_j = S_jk: -S_kj^T if j is eliminated, else stored
    const Opnd Sjk_b = j < k ? opnd_b(tile2_at(a0, m, k, j), m.npad, true, -1.0) : opnd_b(tile2_at(a0, m, j, k), m.npad, false, 1.0);
    copy128(gj_C(scr, m, j), TB2, Sjk_b, sa);
    if (j > k) {
        acc_zero(acc);
        gemm128(acc, opnd_a(tile2_at(a0, m, j, k), m.npad, false, 1.0), Pb, sa, sb);   // new column tile -S_jk P
        acc_store(acc, gj_D(scr, m, j), TB2, -1.0, false);
    }
}

// step k, task (b, i, j), i >= j: trailing update S_ij -= C_i R_j (i, j != k), or the copy of the new
// row tile (i = k > j), column tile (i > k = j) or pivot inverse (i = j = k).
__global__ __launch_bounds__(NT2, 4) void k_gj_update(const int4* __restrict__ tasks, const BlockMeta* __restrict__ meta,
                                                      double* __restrict__ A, double* __restrict__ scr, int64_t pivot_off, int k) {
    __shared__ double sa[2 * KC2 * LS2], sb[2 * KC2 * LS2];
    const int4 t = tasks[blockIdx.x];
    const BlockMeta m = meta[t.x];
    const int i = t.y, j = t.z;
    double* a0 = A + m.mat_off;
    double* gij = tile2_at(a0, m, i, j);
    if (i == k || j == k) {
        const double* src = (i == k && j == k) ? gj_piv(scr, pivot_off, t.x, k) : (i == k) ? gj_R(scr, m, j) : gj_D(scr, m, i);
        copy128(gij, m.npad, opnd_b(src, TB2, false, 1.0), sa);
        return;
    }
    f64x4 acc[4][2];
    acc_zero(acc);
    gemm128(acc, opnd_a(gj_C(scr, m, i), TB2, false, 1.0), opnd_b(gj_R(scr, m, j), TB2, false, 1.0), sa, sb);
    acc_store(acc, gij, m.npad, -1.0, true);
}

// after step k, task (b, k+1, k+1): the pivot inverse of step k+1 from the updated tile, into slot
// (k+1) % 2
__global__ __launch_bounds__(NT2) void k_gj_pivot(const int4* __restrict__ tasks, const BlockMeta* __restrict__ meta,
                                                  double* __restrict__ A, double* __restrict__ scr, int64_t pivot_off, int k,
                                                  int* __restrict__ flags) {
    __shared__ double rowbuf[2 * TB2], colbuf[2 * TB2];
    const int4 t = tasks[blockIdx.x];
    const BlockMeta m = meta[t.x];
    const bool ok = inverse128(tile2_at(A + m.mat_off, m, k + 1, k + 1), m.npad, gj_piv(scr, pivot_off, t.x, k + 1), TB2, rowbuf,
                               colbuf);
    if (!ok && threadIdx.x == 0) flags[t.x] = 1;
}

// the inverse is symmetric: upper tiles (i < j) from the lower ones
__global__ __launch_bounds__(256) void k_mirror(const int4* __restrict__ tasks, const BlockMeta* __restrict__ meta,
                                                double* __restrict__ A) {
    __shared__ double Q[TBK * LDT];
    const int4 t = tasks[blockIdx.x];
    const BlockMeta m = meta[t.x];
    double* a0 = A + m.mat_off;
    tile_load_t(Q, tile_at(a0, m, t.y, t.z), m.npad, 1.0);
    __syncthreads();
    tile_store(Q, tile_at(a0, m, t.z, t.y), m.npad);
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) b[i] = float(a[i]);
}

// --- coarse Galerkin matrix: Y = W R_H^T, then W_H = R_H Y (upper half, mirrored) ------------
// Z = R_H W, by groups of coarse functions.  The coarse dofs are grouped 32 at a time in a
// spatial (Morton) order of their vertices, so a group's supports overlap.  The rows of the union
// of a group's supports are sorted into runs of equal member pattern (the up to 4 members whose
// coefficient is nonzero there: the coarse functions of one coarse triangle, edge or vertex; a
// row with more members appears in several runs).  A one-wave block takes group g = t % ng and the
// 64-column slice t / ng of W: per run, each row is loaded once (eight rows in flight, coalesced)
// and added into 4 slot sums with its coefficients (read through the scalar cache), and at the
// end of the run the slot sums go into the 32 member sums.  Every sum runs in a fixed order:
// bit-reproducible.  Reads of W: the union sizes summed over the groups, about 1.3 N rows (a
// support per coarse dof would read each row about three times).  (W is symmetric, so
// Z^T = W R_H^T.)
constexpr int kZGroup = 32;
constexpr int kZCols = 64;
constexpr int kZSlots = 4;
__global__ __launch_bounds__(64) void k_coarse_Z(const double* __restrict__ W, int64_t ldw, int64_t N, int64_t ng,
                                                 const int32_t* __restrict__ gmem, const int32_t* __restrict__ gmem_ptr,
                                                 const int32_t* __restrict__ grun_ptr, const int32_t* __restrict__ run_row,
                                                 const int4* __restrict__ run_mem, const int32_t* __restrict__ rows,
                                                 const double* __restrict__ coef, double* __restrict__ Z) {
    const int64_t g = blockIdx.x % ng;
    const int64_t c = (blockIdx.x / ng) * kZCols + threadIdx.x;
    const bool valid = c < N;
    double acc[kZGroup];
#pragma unroll
    for (int q = 0; q < kZGroup; ++q) acc[q] = 0.0;
    for (int run = grun_ptr[g]; run < grun_ptr[g + 1]; ++run) {
        const int r0 = run_row[run], r1 = run_row[run + 1];
        double sl[kZSlots] = {0.0, 0.0, 0.0, 0.0};
        constexpr int kU = 8;
        for (int r = r0; r < r1; r += kU) {
            double x[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) x[u] = (valid && r + u < r1) ? W[int64_t(rows[r + u]) * ldw + c] : 0.0;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (r + u < r1) {
                    const double* cf = coef + int64_t(r + u) * kZSlots;
#pragma unroll
                    for (int k = 0; k < kZSlots; ++k) sl[k] = fma(cf[k], x[u], sl[k]);
                }
            }
        }
        const int4 mm = run_mem[run];   // local member of each slot, -1 unused
        const int ms[kZSlots] = {mm.x, mm.y, mm.z, mm.w};
#pragma unroll
        for (int k = 0; k < kZSlots; ++k)
#pragma unroll
            for (int q = 0; q < kZGroup; ++q) acc[q] = (ms[k] == q) ? acc[q] + sl[k] : acc[q];
    }
    if (valid) {
        const int m0 = gmem_ptr[g], nm = gmem_ptr[g + 1] - m0;
#pragma unroll
        for (int q = 0; q < kZGroup; ++q)
            if (q < nm) Z[int64_t(gmem[m0 + q]) * N + c] = acc[q];
    }
}

__global__ void k_coarse_WH(const double* __restrict__ Z, int64_t N, int64_t nH, const int64_t* __restrict__ rp,
                            const int32_t* __restrict__ rc, const double* __restrict__ rv, double shift,
                            double* __restrict__ A, int64_t npad) {
    const int64_t i2 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t i1 = blockIdx.y;
    if (i2 >= npad) return;
    if (i1 >= nH || i2 >= nH) {
        A[i1 * npad + i2] = (i1 == i2) ? 1.0 : 0.0;
        return;
    }
    if (i2 < i1) return;
    // W_H[i1][i2] = sum_e R[i2][e] Z[i1][col_e]
    double s = 0.0;
    const double* z = Z + i1 * N;
    for (int64_t e = rp[i2]; e < rp[i2 + 1]; ++e) s = fma(rv[e], z[rc[e]], s);
    if (i1 == i2) s += shift;
    A[i1 * npad + i2] = s;
    A[i2 * npad + i1] = s;
}

__global__ void k_coarse_pad_rows(double* __restrict__ A, int64_t nH, int64_t npad) {
    // rows nH .. npad-1 of the padded coarse block
    const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t r = nH + blockIdx.y;
    if (c < npad && r < npad) A[r * npad + c] = (r == c) ? 1.0 : 0.0;
}

// --- diagonal wire basket: dinv[e] = 1 / W[d][d] for its dofs d = idx[e]; flag if W_dd <= 0 ---
__global__ void k_wb_diag_setup(const int32_t* __restrict__ idx, int64_t n, const double* __restrict__ W, int64_t ldw,
                                double shift, double* __restrict__ dinv, int* __restrict__ flag) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n) return;
    const int64_t d = idx[e];
    const double w = W[d * ldw + d] + shift;
    if (!(w > 0.0)) *flag = 1;
    dinv[e] = 1.0 / w;
}

// z[c][d] = dinv[e] r[c][d] for the wire-basket dofs d = idx[e] (each dof is in no block then)
__global__ void k_wb_diag_apply(const int32_t* __restrict__ idx, const double* __restrict__ dinv, int64_t n,
                                const double* __restrict__ r, int64_t ld, double* __restrict__ z) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n) return;
    const int64_t off = int64_t(blockIdx.y) * ld + idx[e];
    z[off] = dinv[e] * r[off];
}

// --- apply, step 1: the blocks' right-hand sides, gathered and transposed: Xg[xoff + s][n] ---------
template <typename MT>
__global__ void k_block_gather(const BlockMeta* __restrict__ meta, const int32_t* __restrict__ idx,
                               const double* __restrict__ r, int64_t ld, int kc, MT* __restrict__ xg) {
    const BlockMeta m = meta[blockIdx.y];
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= m.npad * 16) return;
    const int64_t s = e >> 4;
    const int n = int(e & 15);
    xg[m.xoff * 16 + e] = (s < m.n && n < kc) ? MT(r[int64_t(n) * ld + idx[m.idx_off + s]]) : MT(0);
}

// --- apply, step 2: z[idx] = B Xg for a 64-row panel of one block (four 16-row strips) -------------
template <typename MT>
__global__ __launch_bounds__(256) void k_block_apply(const int4* __restrict__ tasks, const BlockMeta* __restrict__ meta,
                                                     const int32_t* __restrict__ idx, const MT* __restrict__ inv,
                                                     const MT* __restrict__ xg, int kc, int64_t ld,
                                                     double* __restrict__ z) {
    using MC = MatrixCore<MT>;
    const int4 t = tasks[blockIdx.x];
    const BlockMeta m = meta[t.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kg = lane >> 4;
    const int64_t row0 = int64_t(t.y) + 16 * wave;
    if (row0 >= m.n) return;
    const int64_t row = row0 + i;                 // < npad: padded rows exist in storage
    // matrix-core sums over chunks of at most 1024 columns, added up in FP64 (for FP32 inverses of
    // large blocks the rounding stays at the level of one chunk)
    double acc64[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t cc = 0; cc < m.npad; cc += 1024) {
        typename MC::V acc = {0, 0, 0, 0};
        strip_mfma<MT, 4>(inv + m.mat_off + row * m.npad, true, cc, min<int64_t>(m.npad, cc + 1024), xg + m.xoff * 16, acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[r] += double(acc[r]);
    }
    if (i < kc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t rr = row0 + MC::out_row(kg, r);
            if (rr < m.n) z[int64_t(i) * ld + idx[m.idx_off + rr]] = acc64[r];
        }
    }
}

// (R_H r)[i][c]: one block per (coarse dof i, column c); threads stride over the fine entries of row
// i of R_H, block sum in a fixed order
__global__ __launch_bounds__(256) void k_restrict(const int64_t* __restrict__ rp, const int32_t* __restrict__ rc,
                                                  const double* __restrict__ rv, int64_t nH,
                                                  const double* __restrict__ r, int64_t ld,
                                                  double* __restrict__ out) {
    __shared__ double red[4];
    const int64_t i = blockIdx.x;
    const int c = blockIdx.y;
    const double* rcol = r + int64_t(c) * ld;
    double acc = 0.0;
    for (int64_t e = rp[i] + threadIdx.x; e < rp[i + 1]; e += blockDim.x) acc = fma(rv[e], rcol[rc[e]], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[int64_t(c) * nH + i] = (red[0] + red[1]) + (red[2] + red[3]);
}

// y = Binv x for the coarse block: one wave per row, lanes over columns
__global__ __launch_bounds__(256) void k_coarse_solve(const double* __restrict__ Binv, int64_t npad, int64_t nH,
                                                      const double* __restrict__ x, int k, double* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (i >= nH) return;
    double acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;
    const double* b = Binv + i * npad;
    for (int64_t j = lane; j < nH; j += 64) {
        const double bij = b[j];
        // columns past k repeat column k - 1 (in bounds, never stored), so the loads need no
        // branches and all issue before the first is used
        double xv[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) xv[c] = x[int64_t(c < k ? c : k - 1) * nH + j];
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = fma(bij, xv[c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        double v = acc[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0 && c < k) y[int64_t(c) * nH + i] = v;
    }
}

// z[c] += R_H^T zc[c]: one thread per (fine dof, column), grid (N / 256, columns)
__global__ void k_prolong_add(const int64_t* __restrict__ tp, const int32_t* __restrict__ tr, const double* __restrict__ tv,
                              int64_t N, const double* __restrict__ zc, int64_t nH, double* __restrict__ z,
                              int64_t ld) {
    const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= N) return;
    const double* u = zc + int64_t(c) * nH;
    double s = 0.0;
    const int64_t e0 = tp[j], e1 = tp[j + 1];
    int64_t e = e0;
    for (; e + 4 <= e1; e += 4) {   // four entries' loads in flight at a time
        double v[4], y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = tv[e + q];
            y[q] = u[tr[e + q]];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) s = fma(v[q], y[q], s);
    }
    for (; e < e1; ++e) s = fma(tv[e], u[tr[e]], s);
    z[int64_t(c) * ld + j] += s;
}

inline unsigned nblk(int64_t n, int per) { return unsigned((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------------------------
// Host: dof classes and the coarse prolongation
// ---------------------------------------------------------------------------------------------
namespace {

struct CoarseCSR {
    int64_t nH = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

// Row (i,j) of R_H: fine coefficients of the coarse jump basis function psi^H_{i,j}.  At a fine
// generalized vertex x_{k,l} the coarse split function phi^H_{i,j} equals lambda^H_i(x_k) when
// the fine sector (k,l) lies in coarse sector j of coarse vertex i, else 0; the jump of the coarse
// function is represented by u_{k,l} - mean_l u_{k,.} on the fine jump basis (l < q_k).
void build_prolongation(const MeshTopo& f, const MeshTopo& c, const int32_t* parent, CoarseCSR& R) {
    const int64_t nt = f.nt;
    // representative side (t, a, s) of every fine sector
    std::vector<int64_t> soff(f.nv + 1, 0);
    for (int64_t v = 0; v < f.nv; ++v) soff[v + 1] = soff[v] + f.q[v];
    std::vector<int64_t> rep(soff[f.nv], -1);
    for (int64_t t = 0; t < nt; ++t)
        for (int a = 0; a < 3; ++a)
            for (int s = 0; s < 2; ++s) {
                int64_t v = f.T[3 * t + a];
                int64_t slot = soff[v] + f.sector[(t * 3 + a) * 2 + s];
                if (rep[slot] < 0) rep[slot] = (t * 3 + a) * 2 + s;
            }
    // entries (coarse dof, fine dof, value), produced per fine vertex on parallel threads; each
    // thread range keeps vertex order, so concatenating the ranges keeps it too
    struct Entry { int32_t i, col; double v; };
    const int64_t grain = 512;
    const int64_t nchunk = (f.nv + grain - 1) / grain;
    std::vector<std::vector<Entry>> part(size_t(std::max<int64_t>(nchunk, 1)));
    FirstFailure ff;
    parallel_for(nchunk, [&](int64_t cb, int64_t ce) {
        struct Acc { int64_t dof; double u[64]; };
        std::vector<Acc> u;
        for (int64_t ch = cb; ch < ce; ++ch) {
            std::vector<Entry>& out = part[size_t(ch)];
            for (int64_t k = ch * grain; k < std::min<int64_t>(f.nv, (ch + 1) * grain); ++k) {
                const int qk = f.q[k];
                if (qk < 2) continue;
                try {
                    if (qk > 64) fail(BEM_E_UNSUPPORTED, "more than 64 sectors at a vertex");
                    u.clear();
                    const double xk[3] = {f.V[3 * k], f.V[3 * k + 1], f.V[3 * k + 2]};
                    for (int l = 0; l < qk; ++l) {
                        const int64_t node = rep[soff[k] + l];
                        const int64_t t = node / 6;
                        const int s = int(node % 2);
                        const int64_t tc = parent[t];
                        double nd = 0;
                        for (int d = 0; d < 3; ++d) nd += f.normal[3 * t + d] * c.normal[3 * tc + d];
                        const int sc = nd > 0 ? s : 1 - s;
                        const double* P0 = &c.V[3 * int64_t(c.T[3 * tc])];
                        const double* P1 = &c.V[3 * int64_t(c.T[3 * tc + 1])];
                        const double* P2 = &c.V[3 * int64_t(c.T[3 * tc + 2])];
                        double e1[3], e2[3], rr[3];
                        for (int d = 0; d < 3; ++d) { e1[d] = P1[d] - P0[d]; e2[d] = P2[d] - P0[d]; rr[d] = xk[d] - P0[d]; }
                        const double g11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
                        const double g12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
                        const double g22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
                        const double b1 = e1[0] * rr[0] + e1[1] * rr[1] + e1[2] * rr[2];
                        const double b2 = e2[0] * rr[0] + e2[1] * rr[1] + e2[2] * rr[2];
                        const double det = g11 * g22 - g12 * g12;
                        const double l1 = (b1 * g22 - b2 * g12) / det, l2 = (g11 * b2 - g12 * b1) / det;
                        const double lam[3] = {1.0 - l1 - l2, l1, l2};
                        double off = 0;   // distance of x_k from the plane of the coarse triangle
                        for (int d = 0; d < 3; ++d) { double pp = rr[d] - l1 * e1[d] - l2 * e2[d]; off += pp * pp; }
                        if (lam[0] < -1e-9 || lam[1] < -1e-9 || lam[2] < -1e-9 || off > 1e-18 * (g11 + g22))
                            fail(BEM_E_INVALID_ARG, "fine triangle " + std::to_string(t) + " is not inside its coarse triangle");
                        for (int ac = 0; ac < 3; ++ac) {
                            if (std::fabs(lam[ac]) < 1e-12) continue;
                            const int64_t i = c.T[3 * tc + ac];
                            const int qi = c.q[i];
                            const int jc = c.sector[(tc * 3 + ac) * 2 + sc];
                            for (int j = 0; j + 1 < qi; ++j) {
                                const double sign = (jc == j) ? 1.0 : (jc == qi - 1 ? -1.0 : 0.0);
                                if (sign == 0.0) continue;
                                const int64_t dof = c.first_dof[i] + j;
                                Acc* a = nullptr;
                                for (auto& x : u) if (x.dof == dof) { a = &x; break; }
                                if (!a) {
                                    u.push_back(Acc{dof, {}});
                                    a = &u.back();
                                    for (int q = 0; q < qk; ++q) a->u[q] = 0.0;
                                }
                                a->u[l] += lam[ac] * sign;
                            }
                        }
                    }
                    std::sort(u.begin(), u.end(), [](const Acc& x, const Acc& y) { return x.dof < y.dof; });
                    for (auto& a : u) {
                        double mean = 0;
                        for (int q = 0; q < qk; ++q) mean += a.u[q];
                        mean /= qk;
                        for (int l = 0; l + 1 < qk; ++l) {
                            const double cv = a.u[l] - mean;
                            if (cv != 0.0) out.push_back(Entry{int32_t(a.dof), int32_t(f.first_dof[k] + l), cv});
                        }
                    }
                } catch (const Failure& x) {
                    ff.record(k, x);
                }
            }
        }
    }, 1);
    ff.rethrow();
    // CSR by coarse dof; within a row the fine dofs come in vertex (hence dof) order
    R.nH = c.N;
    R.ptr.assign(c.N + 1, 0);
    for (auto& pv : part)
        for (auto& e : pv) R.ptr[e.i + 1] += 1;
    for (int64_t i = 0; i < c.N; ++i) R.ptr[i + 1] += R.ptr[i];
    R.col.assign(size_t(R.ptr[c.N]), 0);
    R.val.assign(size_t(R.ptr[c.N]), 0.0);
    std::vector<int64_t> fill(R.ptr.begin(), R.ptr.end() - 1);
    for (auto& pv : part)
        for (auto& e : pv) {
            const int64_t at = fill[e.i]++;
            R.col[size_t(at)] = e.col;
            R.val[size_t(at)] = e.v;
        }
}

// Segment meshes: the same rows of R_H, with the coarse hat function on the coarse segment that
// contains the fine vertex (its two ends' barycentric weights) in place of the triangle's three.
void build_prolongation_2d(const MeshTopo& f, const MeshTopo& c, const int32_t* parent, CoarseCSR& R) {
    const int64_t ns = f.nt;
    std::vector<int64_t> soff(f.nv + 1, 0);
    for (int64_t v = 0; v < f.nv; ++v) soff[v + 1] = soff[v] + f.q[v];
    std::vector<int64_t> rep(soff[f.nv], -1);   // representative side (s, end a, side) per fine sector
    for (int64_t t = 0; t < ns; ++t)
        for (int a = 0; a < 2; ++a)
            for (int sd = 0; sd < 2; ++sd) {
                const int64_t v = f.S[2 * t + a];
                const int64_t slot = soff[v] + f.sector[4 * t + 2 * a + sd];
                if (rep[slot] < 0) rep[slot] = 4 * t + 2 * a + sd;
            }
    struct Entry { int32_t i, col; double v; };
    std::vector<Entry> out;
    struct Acc { int64_t dof; double u[64]; };
    std::vector<Acc> u;
    for (int64_t k = 0; k < f.nv; ++k) {
        const int qk = f.q[k];
        if (qk < 2) continue;
        if (qk > 64) fail(BEM_E_UNSUPPORTED, "more than 64 sectors at a vertex");
        u.clear();
        for (int l = 0; l < qk; ++l) {
            const int64_t node = rep[soff[k] + l];
            const int64_t t = node / 4;
            const int sd = int(node % 2);
            const int64_t tc = parent[t];
            // fine and coarse tangents agree or are opposite; the side labels follow the normal
            const double dot = f.normal[3 * t] * c.normal[3 * tc] + f.normal[3 * t + 1] * c.normal[3 * tc + 1];
            const int sc = dot > 0 ? sd : 1 - sd;
            const double* P0 = &c.V[3 * int64_t(c.S[2 * tc])];
            const double* P1 = &c.V[3 * int64_t(c.S[2 * tc + 1])];
            const double e0 = P1[0] - P0[0], e1 = P1[1] - P0[1];
            const double L2 = e0 * e0 + e1 * e1;
            const double r0 = f.V[3 * k] - P0[0], r1 = f.V[3 * k + 1] - P0[1];
            const double l1 = (r0 * e0 + r1 * e1) / L2;
            const double off = r0 * e1 - r1 * e0;   // distance from the coarse segment's line, times its length
            if (l1 < -1e-9 || l1 > 1.0 + 1e-9 || off * off > 1e-18 * L2 * L2)
                fail(BEM_E_INVALID_ARG, "fine segment " + std::to_string(t) + " is not inside its coarse segment");
            const double lam[2] = {1.0 - l1, l1};
            for (int ac = 0; ac < 2; ++ac) {
                if (std::fabs(lam[ac]) < 1e-12) continue;
                const int64_t i = c.S[2 * tc + ac];
                const int qi = c.q[i];
                const int jc = c.sector[4 * tc + 2 * ac + sc];
                for (int j = 0; j + 1 < qi; ++j) {
                    const double sign = (jc == j) ? 1.0 : (jc == qi - 1 ? -1.0 : 0.0);
                    if (sign == 0.0) continue;
                    const int64_t dof = c.first_dof[i] + j;
                    Acc* a = nullptr;
                    for (auto& x : u) if (x.dof == dof) { a = &x; break; }
                    if (!a) {
                        u.push_back(Acc{dof, {}});
                        a = &u.back();
                        for (int q = 0; q < qk; ++q) a->u[q] = 0.0;
                    }
                    a->u[l] += lam[ac] * sign;
                }
            }
        }
        std::sort(u.begin(), u.end(), [](const Acc& x, const Acc& y) { return x.dof < y.dof; });
        for (auto& a : u) {
            double mean = 0;
            for (int q = 0; q < qk; ++q) mean += a.u[q];
            mean /= qk;
            for (int l = 0; l + 1 < qk; ++l) {
                const double cv = a.u[l] - mean;
                if (cv != 0.0) out.push_back(Entry{int32_t(a.dof), int32_t(f.first_dof[k] + l), cv});
            }
        }
    }
    R.nH = c.N;
    R.ptr.assign(c.N + 1, 0);
    for (auto& e : out) R.ptr[e.i + 1] += 1;
    for (int64_t i = 0; i < c.N; ++i) R.ptr[i + 1] += R.ptr[i];
    R.col.assign(size_t(R.ptr[c.N]), 0);
    R.val.assign(size_t(R.ptr[c.N]), 0.0);
    std::vector<int64_t> fill(R.ptr.begin(), R.ptr.end() - 1);
    for (auto& e : out) {
        const int64_t at = fill[e.i]++;
        R.col[size_t(at)] = e.col;
        R.val[size_t(at)] = e.v;
    }
}

}  // namespace

// Groups of kZGroup coarse dofs for the coarse product: coarse dofs in the Morton order of their
// vertices (10 bits per axis over the coarse mesh's bounding box), cut into consecutive groups.
// Per group, the rows of the union of its functions' fine supports in runs of equal member
// pattern (sorted patterns, rows ascending within a run); a row with more than kZSlots members
// is split over several runs.  Per run its members (local, -1 for an unused slot) and row range;
// per row its fine dof and kZSlots coefficients.
struct CoarseGroups {
    std::vector<int32_t> mem, mem_ptr, run_ptr, run_row, row;
    std::vector<int4> run_mem;
    std::vector<double> coef;
};

void coarse_groups(const MeshTopo& c, const CoarseCSR& R, CoarseGroups& G) {
    const int64_t nH = R.nH;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < c.nv; ++v)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], c.V[3 * v + k]);
            hi[k] = std::max(hi[k], c.V[3 * v + k]);
        }
    auto spread = [](uint64_t x) {   // 10 bits -> every third bit
        x &= 0x3ff;
        x = (x | (x << 16)) & 0x30000ff;
        x = (x | (x << 8)) & 0x300f00f;
        x = (x | (x << 4)) & 0x30c30c3;
        x = (x | (x << 2)) & 0x9249249;
        return x;
    };
    std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(nH));
    for (int64_t i = 0; i < nH; ++i) {
        const int64_t v = c.dof_vertex[i];
        uint64_t code = 0;
        for (int k = 0; k < 3; ++k) {
            const double span = hi[k] > lo[k] ? hi[k] - lo[k] : 1.0;
            const uint64_t qk = uint64_t(std::min(1023.0, std::max(0.0, (c.V[3 * v + k] - lo[k]) / span * 1023.0)));
            code |= spread(qk) << k;
        }
        key[size_t(i)] = {code, int32_t(i)};
    }
    std::sort(key.begin(), key.end());
    const int64_t ng = (nH + kZGroup - 1) / kZGroup;
    G = CoarseGroups{};
    G.mem_ptr.assign(size_t(ng) + 1, 0);
    G.run_ptr.assign(size_t(ng) + 1, 0);
    G.run_row.push_back(0);
    std::vector<std::tuple<int32_t, int32_t, double>> tri;   // (fine dof, member, coefficient)
    // one entry per (row, piece): the piece's members and coefficients (kZSlots each)
    struct Piece { std::array<int32_t, kZSlots> m; int32_t row; std::array<double, kZSlots> v; };
    std::vector<Piece> pieces;
    for (int64_t g = 0; g < ng; ++g) {
        tri.clear();
        pieces.clear();
        const int64_t m0 = g * kZGroup, m1 = std::min<int64_t>(nH, m0 + kZGroup);
        for (int64_t m = m0; m < m1; ++m) {
            const int32_t i = key[size_t(m)].second;
            G.mem.push_back(i);
            for (int64_t e = R.ptr[size_t(i)]; e < R.ptr[size_t(i) + 1]; ++e)
                tri.emplace_back(R.col[size_t(e)], int32_t(m - m0), R.val[size_t(e)]);
        }
        std::sort(tri.begin(), tri.end());
        for (size_t e = 0; e < tri.size();) {
            size_t f = e;
            while (f < tri.size() && std::get<0>(tri[f]) == std::get<0>(tri[e])) ++f;
            for (size_t p0 = e; p0 < f; p0 += kZSlots) {   // members of this row, kZSlots per piece
                Piece pc;
                pc.row = std::get<0>(tri[e]);
                for (int k = 0; k < kZSlots; ++k) {
                    const bool on = p0 + k < f;
                    pc.m[size_t(k)] = on ? std::get<1>(tri[p0 + k]) : -1;
                    pc.v[size_t(k)] = on ? std::get<2>(tri[p0 + k]) : 0.0;
                }
                pieces.push_back(pc);
            }
            e = f;
        }
        std::sort(pieces.begin(), pieces.end(),
                  [](const Piece& x, const Piece& y) { return x.m != y.m ? x.m < y.m : x.row < y.row; });
        for (size_t e = 0; e < pieces.size(); ++e) {
            if (e > 0 && pieces[e].m != pieces[e - 1].m) G.run_row.push_back(int32_t(G.row.size()));
            if (e == 0 || pieces[e].m != pieces[e - 1].m) {
                const auto& mm = pieces[e].m;
                G.run_mem.push_back(make_int4(mm[0], mm[1], mm[2], mm[3]));
            }
            G.row.push_back(pieces[e].row);
            for (int k = 0; k < kZSlots; ++k) G.coef.push_back(pieces[e].v[size_t(k)]);
        }
        if (!pieces.empty()) G.run_row.push_back(int32_t(G.row.size()));
        G.mem_ptr[size_t(g) + 1] = int32_t(G.mem.size());
        G.run_ptr[size_t(g) + 1] = int32_t(G.run_mem.size());
    }
}

void precond_setup_device(bem_precond* M, const int32_t* patch, const double* cV, int64_t ncv, const int32_t* cT,
                          int64_t nct, const int32_t* parent) {
    auto t0 = std::chrono::steady_clock::now();
    bem_problem* p = M->p;
    const MeshTopo& f = p->topo;
    hipStream_t s = p->stream;
    // BEM_TRACE=1: synchronise and print the wall time of each set-up phase to stderr
    const bool trace = std::getenv("BEM_TRACE") != nullptr;
    auto tlast = t0;
    auto mark = [&](const char* what) {
        if (!trace) return;
        HIP_CHECK(hipStreamSynchronize(s));
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "bem-trace precond  %-18s %8.3f ms\n", what, std::chrono::duration<double>(now - tlast).count() * 1e3);
        tlast = now;
    };
    if (!patch) fail(BEM_E_INVALID_ARG, "patch_of_triangle is NULL");

    // ---- dof classes ---------------------------------------------------------------------------
    std::vector<int64_t> vpatch(f.nv, -1);   // -1 unseen, -2 several patches / no patch
    const bool seg = f.dim == 2;              // segment mesh: 2 vertices per element
    const int corners = seg ? 2 : 3;
    for (int64_t t = 0; t < f.nt; ++t)
        for (int a = 0; a < corners; ++a) {
            const int64_t v = seg ? f.S[2 * t + a] : f.T[3 * t + a];
            const int64_t pid = patch[t] < 0 ? -2 : patch[t];
            if (vpatch[v] == -1) vpatch[v] = pid;
            else if (vpatch[v] != pid) vpatch[v] = -2;
        }
    std::map<int64_t, std::vector<int32_t>> faces;
    std::vector<int32_t> wb;
    for (int64_t d = 0; d < f.N; ++d) {
        const int64_t v = f.dof_vertex[d];
        if (vpatch[v] >= 0 && f.q[v] == 2) faces[vpatch[v]].push_back(int32_t(d));
        else wb.push_back(int32_t(d));
    }
    mark("dof classes");
    std::vector<std::vector<int32_t>> blocks;
    for (auto& kv : faces) blocks.push_back(kv.second);
    M->n_faces = int64_t(blocks.size());
    M->n_wb = int64_t(wb.size());
    if (!wb.empty() && !M->wb_diag) blocks.push_back(wb);
    M->max_face = 0;
    for (int64_t b = 0; b < M->n_faces; ++b) M->max_face = std::max<int64_t>(M->max_face, blocks[b].size());
    M->nblocks = int64_t(blocks.size());

    // ---- coarse mesh (its sectors give the coarse dimension; the prolongation is built later,
    //      while the device works on the faces and the wire basket) ----------------------------------
    CoarseCSR R;
    MeshTopo c;
    const bool coarse = M->use_coarse && ncv > 0 && nct > 0;
    if (coarse) {
        if (!cV || !cT || !parent) fail(BEM_E_INVALID_ARG, "coarse mesh arrays missing");
        for (int64_t t = 0; t < f.nt; ++t)
            if (parent[t] < 0 || parent[t] >= nct) fail(BEM_E_INVALID_ARG, "coarse_of_triangle out of range");
        if (seg) analyze_segments(cV, ncv, cT, nct, c);   // cV: ncv x 2, cT: coarse segments nct x 2
        else analyze_mesh(cV, ncv, cT, nct, c);
        M->nH = c.N;
    } else {
        M->nH = 0;
    }
    mark("coarse mesh analysis");

    // ---- block layout (faces, wire basket, then the coarse block) -----------------------------------
    const int64_t nall = M->nblocks + (M->nH > 0 ? 1 : 0);
    std::vector<BlockMeta> meta(nall);
    std::vector<int32_t> idx;
    int64_t moff = 0, xoff = 0;
    for (int64_t b = 0; b < nall; ++b) {
        const int64_t n = (b < M->nblocks) ? int64_t(blocks[b].size()) : M->nH;
        const int64_t npad = ((n + TB2 - 1) / TB2) * TB2;
        meta[b] = {n, npad, int64_t(idx.size()), moff, xoff};
        xoff += npad;
        if (b < M->nblocks) idx.insert(idx.end(), blocks[b].begin(), blocks[b].end());
        moff += npad * npad;
        M->blk_n.push_back(n);
        M->blk_npad.push_back(npad);
        M->blk_idx_off.push_back(meta[b].idx_off);
        M->blk_mat_off.push_back(meta[b].mat_off);
    }
    M->idx_total = int64_t(idx.size());
    M->xg_rows = xoff;
    M->xg = DeviceBuffer(sizeof(double) * 16 * std::max<int64_t>(1, xoff), s);
    M->mat_total = moff;
    M->idx = upload(idx, s);
    M->blk_meta = upload(meta, s);
    DeviceBuffer A(sizeof(double) * std::max<int64_t>(moff, 1), s);
    // Gauss-Jordan scratch: per block its staged tiles (3 x npad x 128), then two pivot tiles each
    const int64_t pivot_off = 3 * xoff * TB2;
    DeviceBuffer scr(sizeof(double) * (pivot_off + nall * 2 * TB2 * TB2), s);
    DeviceBuffer dflags(sizeof(int) * std::max<int64_t>(nall, 1), s);
    HIP_CHECK(hipMemsetAsync(dflags.ptr, 0, sizeof(int) * std::max<int64_t>(nall, 1), s));

    const BlockMeta* dm = M->blk_meta.as<BlockMeta>();

    // ---- every tile task of the set-up, planned on the host and uploaded once.  Two plans: the
    //      faces and the wire basket (problem stream), and the coarse block (second stream, after
    //      its Galerkin matrix) -----------------------------------------------------------------------
    enum Kind { GATHER, GJ_PIVOT0, GJ_ROW, GJ_UPDATE, GJ_PIVOT, MIRROR };
    struct Launch { Kind kind; int param; int64_t off, n; };
    std::vector<int4> all;
    std::vector<Launch> plan_fw, plan_c;
    auto add = [&](std::vector<Launch>& plan, Kind kind, int param, const std::vector<int4>& tl) {
        if (tl.empty()) return;
        plan.push_back({kind, param, int64_t(all.size()), int64_t(tl.size())});
        all.insert(all.end(), tl.begin(), tl.end());
    };
    // 128-wide tiles for the elimination, 64-wide ones for the gather and the mirror
    std::vector<int> ntile(nall), ntile64(nall);
    for (int64_t b = 0; b < nall; ++b) {
        ntile[b] = int(meta[b].npad / TB2);
        ntile64[b] = int(meta[b].npad / TBK);
    }
    auto plan_blocks = [&](std::vector<Launch>& plan, int64_t b0, int64_t b1) {
        int maxT = 0;
        std::vector<int4> tp;
        for (int64_t b = b0; b < b1; ++b) {
            maxT = std::max(maxT, ntile[b]);
            if (ntile[b] > 0) tp.push_back(make_int4(int(b), 0, 0, 0));
        }
        add(plan, GJ_PIVOT0, 0, tp);
        for (int k = 0; k < maxT; ++k) {   // block Gauss-Jordan, all blocks with a step k together
            std::vector<int4> tr, tu, tv;
            for (int64_t b = b0; b < b1; ++b) {   // the next pivot's tile first, then its inversion
                if (k + 1 < ntile[b]) {
                    tu.push_back(make_int4(int(b), k + 1, k + 1, 0));
                    tv.push_back(make_int4(int(b), k + 1, k + 1, 0));
                }
            }
            for (int64_t b = b0; b < b1; ++b) {
                if (k >= ntile[b]) continue;
                for (int j = 0; j < ntile[b]; ++j)
                    if (j != k) tr.push_back(make_int4(int(b), k, j, 0));
                for (int i = 0; i < ntile[b]; ++i)
                    for (int j = 0; j <= i; ++j)
                        if (!(i == k + 1 && j == k + 1)) tu.push_back(make_int4(int(b), i, j, 0));
            }
            add(plan, GJ_ROW, k, tr);
            add(plan, GJ_UPDATE, k, tu);
            add(plan, GJ_PIVOT, k, tv);
        }
        std::vector<int4> tm;
        for (int64_t b = b0; b < b1; ++b)
            for (int i = 1; i < ntile64[b]; ++i)
                for (int j = 0; j < i; ++j) tm.push_back(make_int4(int(b), i, j, 0));
        add(plan, MIRROR, 0, tm);
    };
    {
        std::vector<int4> tl;
        for (int64_t b = 0; b < M->nblocks; ++b)
            for (int i = 0; i < ntile64[b]; ++i)
                for (int j = 0; j < ntile64[b]; ++j) tl.push_back(make_int4(int(b), i, j, 0));
        add(plan_fw, GATHER, 0, tl);
    }
    plan_blocks(plan_fw, 0, M->nblocks);
    plan_blocks(plan_c, M->nblocks, nall);
    DeviceBuffer dtasks = upload(all, s);
    const int4* T0 = dtasks.as<int4>();
    mark("layout+plan+upload");
    auto run = [&](const Launch& L, hipStream_t st) {
        const int4* d = T0 + L.off;
        const dim3 g(unsigned(L.n)), bl(256);
        switch (L.kind) {
            case GATHER: hipLaunchKernelGGL(k_gather, g, bl, 0, st, d, dm, M->idx.as<int32_t>(), p->W64.as<double>(), p->ldw, M->diag_shift, A.as<double>()); break;
            case GJ_PIVOT0: hipLaunchKernelGGL(k_gj_pivot0, g, dim3(NT2), 0, st, d, dm, A.as<double>(), scr.as<double>(), pivot_off, dflags.as<int>()); break;
            case GJ_ROW: hipLaunchKernelGGL(k_gj_row, g, dim3(NT2), 0, st, d, dm, A.as<double>(), scr.as<double>(), pivot_off, L.param); break;
            case GJ_UPDATE: hipLaunchKernelGGL(k_gj_update, g, dim3(NT2), 0, st, d, dm, A.as<double>(), scr.as<double>(), pivot_off, L.param); break;
            case GJ_PIVOT: hipLaunchKernelGGL(k_gj_pivot, g, dim3(NT2), 0, st, d, dm, A.as<double>(), scr.as<double>(), pivot_off, L.param, dflags.as<int>()); break;
            case MIRROR: hipLaunchKernelGGL(k_mirror, g, bl, 0, st, d, dm, A.as<double>()); break;
        }
        HIP_CHECK(hipGetLastError());
    };
    // the coarse block's work (second stream) starts after the layout uploads queued so far
    hipStream_t s2 = s;
    if (M->nH > 0) {
        if (!p->aux_stream) p->aux_stream = acquire_stream(p->ctx);
        s2 = p->aux_stream;
        hipEvent_t ready;
        HIP_CHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        const hipError_t e1 = hipEventRecord(ready, s);
        const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s2, ready, 0) : e1;
        (void)hipEventDestroy(ready);
        HIP_CHECK(e2);
    }
    // faces and wire basket: all of their work is queued now.  (Queueing the coarse path ahead of
    // most of it was slower: the memory-bound coarse product then takes the CUs that the
    // latency-bound elimination steps wait for.)
    for (const Launch& L : plan_fw) run(L, s);

    // coarse Galerkin block on the second stream, while the first one eliminates
    DeviceBuffer Z, d_gmem, d_gmem_ptr, d_grow_ptr, d_grow, d_gcoef, d_grun_row, d_grun_mem;
    CoarseGroups grp;   // host sides of the group uploads: they must outlive the copies
    std::vector<int64_t> tp;   // host sides of the coarse uploads: they must outlive the copies
    std::vector<int32_t> trow;
    std::vector<double> tval;
    if (M->nH > 0) {
        const auto hp0 = std::chrono::steady_clock::now();
        if (seg) build_prolongation_2d(f, c, parent, R);
        else build_prolongation(f, c, parent, R);
        if (trace)
            std::fprintf(stderr, "bem-trace precond  %-18s %8.3f ms (host only)\n", "prolongation build",
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - hp0).count() * 1e3);
        mark("prolongation");
        // transposed CSR (fine dof -> coarse dofs)
        tp.assign(size_t(f.N) + 1, 0);
        for (int32_t cidx : R.col) ++tp[cidx + 1];
        for (int64_t j = 0; j < f.N; ++j) tp[j + 1] += tp[j];
        trow.assign(R.col.size(), 0);
        tval.assign(R.col.size(), 0.0);
        std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
        for (int64_t i = 0; i < R.nH; ++i)
            for (int64_t e = R.ptr[i]; e < R.ptr[i + 1]; ++e) {
                int64_t pos = fill[R.col[e]]++;
                trow[pos] = int32_t(i);
                tval[pos] = R.val[e];
            }
        M->rh_ptr = upload(R.ptr, s2);
        M->rh_col = upload(R.col, s2);
        M->rh_val = upload(R.val, s2);
        M->rht_ptr = upload(tp, s2);
        M->rht_row = upload(trow, s2);
        M->rht_val = upload(tval, s2);
        Z = DeviceBuffer(sizeof(double) * std::max<int64_t>(1, f.N * M->nH), s2);
        coarse_groups(c, R, grp);
        const int64_t ng = int64_t(grp.mem_ptr.size()) - 1;
        d_gmem = upload(grp.mem, s2);
        d_gmem_ptr = upload(grp.mem_ptr, s2);
        d_grow_ptr = upload(grp.run_ptr, s2);
        d_grow = upload(grp.row, s2);
        d_gcoef = upload(grp.coef, s2);
        d_grun_row = upload(grp.run_row, s2);
        d_grun_mem = upload(grp.run_mem, s2);
        const int64_t zblocks = int64_t(nblk(f.N, kZCols)) * ng;
        hipLaunchKernelGGL(k_coarse_Z, dim3(unsigned(zblocks)), dim3(64), 0, s2, p->W64.as<double>(), p->ldw, f.N, ng,
                           d_gmem.as<int32_t>(), d_gmem_ptr.as<int32_t>(), d_grow_ptr.as<int32_t>(), d_grun_row.as<int32_t>(),
                           d_grun_mem.as<int4>(), d_grow.as<int32_t>(), d_gcoef.as<double>(), Z.as<double>());
        HIP_CHECK(hipGetLastError());
        const BlockMeta& cm = meta[nall - 1];
        double* Ac = A.as<double>() + cm.mat_off;
        hipLaunchKernelGGL(k_coarse_WH, dim3(nblk(cm.npad, 256), unsigned(M->nH)), dim3(256), 0, s2, Z.as<double>(), f.N, M->nH,
                           M->rh_ptr.as<int64_t>(), M->rh_col.as<int32_t>(), M->rh_val.as<double>(), M->diag_shift, Ac, cm.npad);
        HIP_CHECK(hipGetLastError());
        if (cm.npad > M->nH) {
            hipLaunchKernelGGL(k_coarse_pad_rows, dim3(nblk(cm.npad, 256), unsigned(cm.npad - M->nH)), dim3(256), 0, s2, Ac, M->nH, cm.npad);
            HIP_CHECK(hipGetLastError());
        }
        for (const Launch& L : plan_c) run(L, s2);
    }
    if (M->nH > 0) HIP_CHECK(hipStreamSynchronize(s2));
    HIP_CHECK(hipStreamSynchronize(s));
    mark("factor+invert");
    std::vector<int> flags(nall);
    HIP_CHECK(hipMemcpyAsync(flags.data(), dflags.ptr, sizeof(int) * nall, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int64_t b = 0; b < nall; ++b)
        if (flags[b]) fail(BEM_E_NOT_SPD, "preconditioner block " + std::to_string(b) + " is not positive definite");
    if (M->wb_diag && M->n_wb > 0) {
        M->wb_idx = upload(wb, s);
        M->wb_dinv = DeviceBuffer(sizeof(double) * M->n_wb, s);
        DeviceBuffer wflag(sizeof(int), s);
        HIP_CHECK(hipMemsetAsync(wflag.ptr, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_wb_diag_setup, dim3(nblk(M->n_wb, 256)), dim3(256), 0, s, M->wb_idx.as<int32_t>(), M->n_wb,
                           p->W64.as<double>(), p->ldw, M->diag_shift, M->wb_dinv.as<double>(), wflag.as<int>());
        HIP_CHECK(hipGetLastError());
        int hf = 0;
        HIP_CHECK(hipMemcpyAsync(&hf, wflag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (hf) fail(BEM_E_NOT_SPD, "a diagonal entry of W on the wire basket is not positive");
    }
    M->inv64 = std::move(A);
    if (M->fp32) {
        M->inv32 = DeviceBuffer(sizeof(float) * std::max<int64_t>(moff, 1), s);
        hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(256), 0, s, M->inv64.as<double>(), M->inv32.as<float>(), moff);
        HIP_CHECK(hipGetLastError());
    }
    // the coarse inverse lives in inv64 as the last block

    // ---- apply tasks: 64-row panels of the face / wire-basket blocks ------------------------------
    std::vector<int4> at;
    for (int64_t b = 0; b < M->nblocks; ++b)
        for (int64_t r0 = 0; r0 < meta[b].n; r0 += 64)
            at.push_back(make_int4(int(b), int(r0), int(std::min<int64_t>(64, meta[b].n - r0)), 0));
    M->ntasks = int64_t(at.size());
    M->max_npad = 0;
    for (int64_t b = 0; b < M->nblocks; ++b) M->max_npad = std::max<int64_t>(M->max_npad, meta[b].npad);
    M->tasks = upload(at, s);
    HIP_CHECK(hipStreamSynchronize(s));
    M->bytes = int64_t(M->inv64.bytes + M->inv32.bytes + M->idx.bytes + M->rh_val.bytes * 3 + M->wb_idx.bytes +
                       M->wb_dinv.bytes);
    mark("fp32+apply tasks");
    M->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

int64_t precond_scratch_size(const bem_precond* m, int k) { return 2 * std::max<int64_t>(1, m->nH) * k; }

void precond_apply_device(const bem_precond* M, bool fp32, const double* r, int64_t ld, int k, double* z,
                          hipStream_t s, double* scratch) {
    const BlockMeta* dm = M->blk_meta.as<BlockMeta>();
    const bem_problem* p = M->p;
    for (int c0 = 0; c0 < k; c0 += 16) {
        const int kc = std::min(16, k - c0);
        const double* rc = r + int64_t(c0) * ld;
        double* zc = z + int64_t(c0) * ld;
        if (M->ntasks > 0) {
            unsigned gx = unsigned((M->max_npad * 16 + 255) / 256);
            if (fp32 && M->inv32.ptr) {
                float* xg = M->xg.as<float>();
                hipLaunchKernelGGL(k_block_gather<float>, dim3(gx, unsigned(M->nblocks)), dim3(256), 0, s, dm, M->idx.as<int32_t>(), rc, ld, kc, xg);
                hipLaunchKernelGGL(k_block_apply<float>, dim3(unsigned(M->ntasks)), dim3(256), 0, s, M->tasks.as<int4>(), dm,
                                   M->idx.as<int32_t>(), M->inv32.as<float>(), xg, kc, ld, zc);
            } else {
                double* xg = M->xg.as<double>();
                hipLaunchKernelGGL(k_block_gather<double>, dim3(gx, unsigned(M->nblocks)), dim3(256), 0, s, dm, M->idx.as<int32_t>(), rc, ld, kc, xg);
                hipLaunchKernelGGL(k_block_apply<double>, dim3(unsigned(M->ntasks)), dim3(256), 0, s, M->tasks.as<int4>(), dm,
                                   M->idx.as<int32_t>(), M->inv64.as<double>(), xg, kc, ld, zc);
            }
            HIP_CHECK(hipGetLastError());
        }
        if (M->wb_diag && M->n_wb > 0) {
            hipLaunchKernelGGL(k_wb_diag_apply, dim3(nblk(M->n_wb, 256), unsigned(kc)), dim3(256), 0, s,
                               M->wb_idx.as<int32_t>(), M->wb_dinv.as<double>(), M->n_wb, rc, ld, zc);
            HIP_CHECK(hipGetLastError());
        }
        if (M->nH > 0) {
            const int64_t nH = M->nH;
            double* rcoarse = scratch;
            double* zcoarse = scratch + nH * kc;
            hipLaunchKernelGGL(k_restrict, dim3(unsigned(nH), unsigned(kc)), dim3(256), 0, s, M->rh_ptr.as<int64_t>(),
                               M->rh_col.as<int32_t>(), M->rh_val.as<double>(), nH, rc, ld, rcoarse);
            const int64_t cb = M->nblocks;
            const double* Binv = M->inv64.as<double>() + M->blk_mat_off[cb];
            hipLaunchKernelGGL(k_coarse_solve, dim3(nblk(nH, 4)), dim3(256), 0, s, Binv, M->blk_npad[cb], nH, rcoarse, kc, zcoarse);
            hipLaunchKernelGGL(k_prolong_add, dim3(nblk(p->N, 256), unsigned(kc)), dim3(256), 0, s, M->rht_ptr.as<int64_t>(),
                               M->rht_row.as<int32_t>(), M->rht_val.as<double>(), p->N, zcoarse, nH, zc, ld);
            HIP_CHECK(hipGetLastError());
        }
    }
}

}  // namespace bem
