// Dense assembly of the hypersingular Galerkin matrix in surface-curl form (paper: Section 4.3,
// eq. eval_a_phiij with Cor. corW):
//
//   W_{d,d'} = sum_{T,T'} I(T,T') J_{T,d} . J_{T',d'},   I(T,T') = 1/(4 pi) int_T int_T' |x-y|^{-1},
//   J_{T,d} = c_{T,a,d} (x_{a+1} - x_{a+2}) / (2|T|)   (dof d sits at corner a of T).
//
// Pipeline (all on the device):
//   k_geometry      per triangle: unit normal, area, the 7 Gauss points and area-weights
//   k_jump_vectors  per (dof, triangle) incidence: J_{T,d}
//   k_group_bounds  per group of 16 triangles: bounding sphere of their Gauss points
//   k_col_records   per triangle: its Gauss points about its group's centre, scaled by 1/w^2
//   k_far           7x7 product rule for every pair in 64x64 triangle tiles above the diagonal;
//                   each lane keeps its row triangle's Gauss points in registers while the wave
//                   walks the tile's column triangles, whose data come in through scalar loads;
//                   separated groups use a centred form of |x - y|^2 (fewer instructions)
//   k_near_*        Duffy-regularised Gauss-Legendre rules for pairs sharing a triangle, an edge
//                   or a vertex (overwrite the far-rule values of those pairs)
//   k_contract      W = sum over the stars of the two dofs, upper triangle, mirrored
//
// The near rules here are the 4-D Duffy rules of the oracle with the radial variable (and, for
// the coincident and edge cases, the anchor variables) integrated exactly: for the kernel
// 1/|x-y| the integrand is a polynomial of degree <= 2 in those variables, which Gauss-Legendre
// integrates exactly from 2 points on, so dropping them changes nothing but rounding.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <memory>
#include <thread>

#include "internal.h"

namespace bem {

namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;
constexpr int kGeo = 28;   // 21 Gauss-point coordinates + 7 area-weights per triangle
constexpr int kTile = 64;

__device__ __forceinline__ double rsqrt_refined(double x) {
    // hardware reciprocal square root (about 2^-23 relative error) and one Newton step
    double y = __builtin_amdgcn_rsq(x);
    double t = y * y;
    double e = fma(-0.5 * x, t, 0.5);
    return fma(y, e, y);
}

__global__ void k_geometry(const double* __restrict__ V, const int32_t* __restrict__ T, int64_t nt,
                           const double* __restrict__ bary7, const double* __restrict__ w7,
                           double* __restrict__ geo, double* __restrict__ normal, double* __restrict__ area) {
    int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    double x[3][3];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) x[a][k] = V[3 * int64_t(T[3 * t + a]) + k];
    double e1[3], e2[3], c[3];
    for (int k = 0; k < 3; ++k) { e1[k] = x[1][k] - x[0][k]; e2[k] = x[2][k] - x[0][k]; }
    c[0] = e1[1] * e2[2] - e1[2] * e2[1];
    c[1] = e1[2] * e2[0] - e1[0] * e2[2];
    c[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double tw = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int k = 0; k < 3; ++k) normal[3 * t + k] = c[k] / tw;
    double ar = 0.5 * tw;
    area[t] = ar;
    double* g = geo + t * kGeo;
    for (int p = 0; p < 7; ++p) {
        for (int k = 0; k < 3; ++k)
            g[3 * p + k] = bary7[3 * p] * x[0][k] + bary7[3 * p + 1] * x[1][k] + bary7[3 * p + 2] * x[2][k];
        g[21 + p] = ar * w7[p];
    }
}

__global__ void k_jump_vectors(const double* __restrict__ V, const int32_t* __restrict__ T,
                               const int32_t* __restrict__ ent_tri, const int8_t* __restrict__ ent_corner,
                               const int8_t* __restrict__ ent_c, const double* __restrict__ area,
                               int64_t ne, double* __restrict__ J) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= ne) return;
    int64_t t = ent_tri[e];
    int a = ent_corner[e];
    int32_t v1 = T[3 * t + (a + 1) % 3], v2 = T[3 * t + (a + 2) % 3];
    double s = double(ent_c[e]) / (2.0 * area[t]);
    for (int k = 0; k < 3; ++k) J[3 * e + k] = s * (V[3 * int64_t(v1) + k] - V[3 * int64_t(v2) + k]);
}

// renumbered device copies of the mesh (see renumber_mesh_device)
__global__ void k_renumber_mesh(const double* __restrict__ V, const int32_t* __restrict__ T, int64_t nv, int64_t nt,
                                const int32_t* __restrict__ vert_user, const int32_t* __restrict__ vert_int,
                                const int32_t* __restrict__ tri_user, double* __restrict__ Vout, int32_t* __restrict__ Tout) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nv)
        for (int c = 0; c < 3; ++c) Vout[3 * i + c] = V[3 * int64_t(vert_user[i]) + c];
    if (i < nt)
        for (int a = 0; a < 3; ++a) Tout[3 * i + a] = vert_int[T[3 * int64_t(tri_user[i]) + a]];
}

// ---------------------------------------------------------------------------------------------
// Far field.  For the Gauss points x (row triangle) and y (column triangle, area-weight w), centred
// on a point c with u = -2 (x - c), alpha = |x - c|^2 and v = y - c,
//
//   |x - y|^2 / w^2 = alpha (1/w^2) + |v|^2/w^2 + u . (v/w^2),
//
// so with the column point stored as the record (v/w^2, 1/w^2, |v|^2/w^2) one fused multiply-add
// and three more give |x - y|^2 / w^2, whose reciprocal square root is w / |x - y| itself: the
// column weight costs nothing and the distance costs four instructions instead of six.  With the
// Newton step y (3 - s y^2) / 2 and the sum, an evaluation is 7 FP64 instructions and the
// reciprocal square root (a quarter-rate instruction), against 10 and the same root for the
// differences x - y.
//
// Rounding: the terms are bounded by (|x - c| + |y - c|)^2, so the relative error of |x - y|^2
// grows like ((|x - c| + |y - c|) / |x - y|)^2.  c is the centre of the column triangle's group of
// 16 (consecutive triangles); a group of columns takes this form only if its centre is at least
// kSep (rho_R + rho_C) from the centre of the row tile (rho the radii of the Gauss points about
// the centres), which bounds that ratio by (kSep + 1) / (kSep - 1): 11 for the default kSep = 1.2,
// at worst about 121 ulp of |x - y|^2, 1.3e-14 relative (kSep is a launch parameter, at least
// 1.1: ratio 21, 1e-13).  Closer groups take the differences.  Pairs that share a vertex are
// overwritten by the near rules in either case.
// ---------------------------------------------------------------------------------------------
constexpr int kGrp = 16;
constexpr int kRec = 35;   // 7 points x (v/w^2, 1/w^2, |v|^2/w^2)

// per group of 16 consecutive triangles: centre of the bounding box of their Gauss points, and the
// largest distance of one of those points from it
__global__ void k_group_bounds(const double* __restrict__ geo, int32_t nt, double* __restrict__ gb) {
    const int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t ng = (int64_t(nt) + kGrp - 1) / kGrp;
    if (g >= ng) return;
    const int64_t t0 = g * kGrp, t1 = min<int64_t>(nt, t0 + kGrp);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t t = t0; t < t1; ++t)
        for (int p = 0; p < 7; ++p)
            for (int k = 0; k < 3; ++k) {
                const double v = geo[t * kGeo + 3 * p + k];
                lo[k] = fmin(lo[k], v);
                hi[k] = fmax(hi[k], v);
            }
    double c[3], r2 = 0.0;
    for (int k = 0; k < 3; ++k) c[k] = 0.5 * (lo[k] + hi[k]);
    for (int64_t t = t0; t < t1; ++t)
        for (int p = 0; p < 7; ++p) {
            double d2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double d = geo[t * kGeo + 3 * p + k] - c[k];
                d2 = fma(d, d, d2);
            }
            r2 = fmax(r2, d2);
        }
    gb[4 * g] = c[0];
    gb[4 * g + 1] = c[1];
    gb[4 * g + 2] = c[2];
    gb[4 * g + 3] = sqrt(r2) * (1.0 + 1e-12);
}

// per triangle: its 7 column records about the centre of its group
__global__ void k_col_records(const double* __restrict__ geo, const double* __restrict__ gb, int32_t nt,
                              double* __restrict__ rec) {
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    const double* c = gb + 4 * (t / kGrp);
    for (int q = 0; q < 7; ++q) {
        const double w = geo[t * kGeo + 21 + q];
        const double iw2 = 1.0 / (w * w);
        const double v0 = geo[t * kGeo + 3 * q] - c[0], v1 = geo[t * kGeo + 3 * q + 1] - c[1],
                     v2 = geo[t * kGeo + 3 * q + 2] - c[2];
        double* r = rec + t * kRec + 5 * q;
        r[0] = v0 * iw2;
        r[1] = v1 * iw2;
        r[2] = v2 * iw2;
        r[3] = iw2;
        r[4] = fma(v0, v0, fma(v1, v1, v2 * v2)) * iw2;
    }
}

// One wave per 64x64 tile (rb <= cb); 4 waves per block.  Lane t keeps its row triangle's 7 Gauss
// points in registers; the wave walks the tile's column triangles in chunks of 16 (one group),
// whose data arrive through scalar loads, each chunk in the centred form above or by differences.
// Results go out per chunk: row tp of I directly (64 consecutive entries), and row t of I through
// an LDS transpose so that each store instruction writes eight complete 128-byte row segments
// instead of 64 scattered 8-byte pieces.
constexpr int kChunk = kGrp;

__global__ __launch_bounds__(256) void k_far(const double* __restrict__ geo, const double* __restrict__ gb,
                                             const double* __restrict__ rec, int32_t nt, int64_t ld,
                                             const int2* __restrict__ tiles, int64_t ntiles, double kSep,
                                             double* __restrict__ I) {
    __shared__ double stage[4][kTile][kChunk + 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t tile = int64_t(blockIdx.x) * 4 + wave;
    if (tile >= ntiles) return;
    const int2 tc = tiles[tile];
    const int rb = __builtin_amdgcn_readfirstlane(tc.x);
    const int cb = __builtin_amdgcn_readfirstlane(tc.y);
    const int t = rb * kTile + lane;
    const bool valid = t < nt;
    const double* g = geo + int64_t(valid ? t : 0) * kGeo;
    // bounding sphere of the row tile's Gauss points, from those of its (up to 4) groups
    double cR[3], rhoR = 0.0;
    {
        const int g0 = rb * (kTile / kGrp), g1 = min((nt + kGrp - 1) / kGrp, g0 + kTile / kGrp);
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int gg = g0; gg < g1; ++gg)
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], gb[4 * gg + k] - gb[4 * gg + 3]);
                hi[k] = fmax(hi[k], gb[4 * gg + k] + gb[4 * gg + 3]);
            }
        for (int k = 0; k < 3; ++k) cR[k] = 0.5 * (lo[k] + hi[k]);
        for (int gg = g0; gg < g1; ++gg) {
            const double d0 = gb[4 * gg] - cR[0], d1 = gb[4 * gg + 1] - cR[1], d2 = gb[4 * gg + 2] - cR[2];
            rhoR = fmax(rhoR, sqrt(fma(d0, d0, fma(d1, d1, d2 * d2))) + gb[4 * gg + 3]);
        }
        rhoR *= 1.0 + 1e-12;
    }
    const int c0 = cb * kTile;
    const int c1 = min(c0 + kTile, nt);
    // row stride ld is a multiple of 8 doubles, so the paired stores below are 16-byte aligned
    // full off-diagonal tiles use the staged stores; diagonal and ragged tiles store directly
    const bool staged = (rb != cb) && (c1 - c0 == kTile) && (rb * kTile + kTile <= nt);
    // I(t, tp) for the lane's row t: row tp of I directly; row t later, from the staging tile
    auto put = [&](int j, int tp, double v) {
        if (staged) {
            I[int64_t(tp) * ld + t] = v;   // row tp: 64 consecutive entries
            stage[wave][lane][j] = v;
        } else if (valid && tp < c1 && (rb != cb || t < tp)) {
            I[int64_t(tp) * ld + t] = v;
            I[int64_t(t) * ld + tp] = v;
        }
    };
    for (int j0 = c0; j0 < c1; j0 += kChunk) {
        // the row triangle's points are read again per chunk (cache hits), so that only one of
        // the two forms' register sets is live at a time
        double pw[7];
#pragma unroll
        for (int p = 0; p < 7; ++p) pw[p] = 0.5 * g[21 + p];   // the 1/2 of the Newton step (exact)
        const double* gC = gb + 4 * (j0 / kGrp);
        const double e0 = gC[0] - cR[0], e1 = gC[1] - cR[1], e2 = gC[2] - cR[2];
        const double sep = kSep * (rhoR + gC[3]);
        if (fma(e0, e0, fma(e1, e1, e2 * e2)) >= sep * sep) {
            // centred form about the group centre c: u = -2 (x - c), alpha = |x - c|^2
            double ux[7], uy[7], uz[7], al[7];
#pragma unroll
            for (int p = 0; p < 7; ++p) {
                const double a0 = g[3 * p] - gC[0], a1 = g[3 * p + 1] - gC[1], a2 = g[3 * p + 2] - gC[2];
                ux[p] = -2.0 * a0;
                uy[p] = -2.0 * a1;
                uz[p] = -2.0 * a2;
                al[p] = fma(a0, a0, fma(a1, a1, a2 * a2));
            }
#pragma unroll 1
            for (int j = 0; j < kChunk; ++j) {
                const int tp = j0 + j;
                double acc = 0.0;
                if (tp < c1) {
                    const double* h = rec + int64_t(tp) * kRec;
#pragma unroll
                    for (int p = 0; p < 7; ++p) {
                        double sacc = 0.0;
#pragma unroll
                        for (int q = 0; q < 7; ++q) {
                            // s = |x - y|^2 / w^2 and 1/sqrt(s) = w / |x - y|, one Newton step from
                            // the hardware estimate y: y (3 - s y^2) / 2
                            const double* r = h + 5 * q;
                            const double s2 = fma(ux[p], r[0], fma(uy[p], r[1], fma(uz[p], r[2], fma(al[p], r[3], r[4]))));
                            const double y = __builtin_amdgcn_rsq(s2);
                            sacc = fma(y, fma(-s2, y * y, 3.0), sacc);
                        }
                        acc = fma(pw[p], sacc, acc);
                    }
                }
                put(j, tp, acc * kInv4Pi);
            }
        } else {
            double px[7], py[7], pz[7];
#pragma unroll
            for (int p = 0; p < 7; ++p) {
                px[p] = g[3 * p];
                py[p] = g[3 * p + 1];
                pz[p] = g[3 * p + 2];
            }
#pragma unroll 1
            for (int j = 0; j < kChunk; ++j) {
                const int tp = j0 + j;
                double acc = 0.0;
                if (tp < c1) {
                    const double* h = geo + int64_t(tp) * kGeo;
#pragma unroll
                    for (int q = 0; q < 7; ++q) {
                        const double yx = h[3 * q], yy = h[3 * q + 1], yz = h[3 * q + 2];
                        double sacc = 0.0;
#pragma unroll
                        for (int p = 0; p < 7; ++p) {
                            const double dx = px[p] - yx, dy = py[p] - yy, dz = pz[p] - yz;
                            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                            // 1/r = y (3 - r2 y^2) / 2 after one Newton step from the hardware estimate y
                            const double y = __builtin_amdgcn_rsq(r2);
                            sacc = fma(pw[p] * y, fma(-r2, y * y, 3.0), sacc);
                        }
                        acc = fma(h[21 + q], sacc, acc);
                    }
                }
                put(j, tp, acc * kInv4Pi);
            }
        }
        if (staged) {
            __builtin_amdgcn_wave_barrier();   // stage[wave] is private to this wave; order write -> read
            // row t: lanes 8r .. 8r+7 write row (8 pass + r) of the tile, 16 bytes each
#pragma unroll
            for (int pass = 0; pass < 8; ++pass) {
                const int row = pass * 8 + (lane >> 3);
                const int col = (lane & 7) * 2;
                const double2 v = make_double2(stage[wave][row][col], stage[wave][row][col + 1]);
                *reinterpret_cast<double2*>(I + int64_t(rb * kTile + row) * ld + j0 + col) = v;
            }
            __builtin_amdgcn_wave_barrier();   // reads done before the next chunk overwrites stage
        }
    }
}

// Panel form of the far-field pass: I_P[r][c - col0] for the rows r of a list of triangles (the
// panel's rows) and the columns c in [col0, nt), col0 a multiple of 16.  One wave per tile of 64
// listed rows x 64 columns: as in k_far, lane l keeps listed row 64 rb + l in registers and walks
// the tile's columns in groups of 16, each in the centred form or by differences (the separation
// test uses the bounding sphere of the tile's rows, reduced across the wave), and each group's
// 64 x 16 block goes out through an LDS transpose as 128-byte row segments.
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(256) void k_far_rect(const double* __restrict__ geo, const double* __restrict__ gb,
                                                  const double* __restrict__ rec, int32_t nt,
                                                  const int32_t* __restrict__ rows, int64_t nrows, int64_t col0, int64_t ld,
                                                  const int2* __restrict__ tiles, int64_t ntiles, double kSep,
                                                  double* __restrict__ I) {
    __shared__ double stage[4][kTile][kChunk + 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t tile = int64_t(blockIdx.x) * 4 + wave;
    if (tile >= ntiles) return;
    const int2 tc = tiles[tile];
    const int rb = __builtin_amdgcn_readfirstlane(tc.x);
    const int cb = __builtin_amdgcn_readfirstlane(tc.y);
    const int64_t r = int64_t(rb) * kTile + lane;   // listed row of this lane
    const bool valid = r < nrows;
    const double* g = geo + int64_t(rows[valid ? r : 0]) * kGeo;
    // bounding sphere of the tile's rows
    double cR[3], rhoR = 0.0;
    {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (valid)
            for (int p = 0; p < 7; ++p)
                for (int k = 0; k < 3; ++k) {
                    lo[k] = fmin(lo[k], g[3 * p + k]);
                    hi[k] = fmax(hi[k], g[3 * p + k]);
                }
        for (int k = 0; k < 3; ++k) cR[k] = 0.5 * (wave_min(lo[k]) + wave_max(hi[k]));
        double d2 = 0.0;
        if (valid)
            for (int p = 0; p < 7; ++p) {
                const double a0 = g[3 * p] - cR[0], a1 = g[3 * p + 1] - cR[1], a2 = g[3 * p + 2] - cR[2];
                d2 = fmax(d2, fma(a0, a0, fma(a1, a1, a2 * a2)));
            }
        rhoR = sqrt(wave_max(d2)) * (1.0 + 1e-12);
    }
    const int64_t c0 = col0 + int64_t(cb) * kTile;
    const int64_t c1 = min<int64_t>(c0 + kTile, nt);
    const bool staged = (c1 - c0 == kTile) && (int64_t(rb) * kTile + kTile <= nrows);
    auto put = [&](int j, int64_t tp, double v) {
        if (staged) stage[wave][lane][j] = v;
        else if (valid && tp < c1) I[r * ld + (tp - col0)] = v;
    };
    for (int64_t j0 = c0; j0 < c1; j0 += kChunk) {
        double pw[7];
#pragma unroll
        for (int p = 0; p < 7; ++p) pw[p] = 0.5 * g[21 + p];   // the 1/2 of the Newton step (exact)
        const double* gC = gb + 4 * (j0 / kGrp);
        const double e0 = gC[0] - cR[0], e1 = gC[1] - cR[1], e2 = gC[2] - cR[2];
        const double sep = kSep * (rhoR + gC[3]);
        if (fma(e0, e0, fma(e1, e1, e2 * e2)) >= sep * sep) {
            double ux[7], uy[7], uz[7], al[7];
#pragma unroll
            for (int p = 0; p < 7; ++p) {
                const double a0 = g[3 * p] - gC[0], a1 = g[3 * p + 1] - gC[1], a2 = g[3 * p + 2] - gC[2];
                ux[p] = -2.0 * a0;
                uy[p] = -2.0 * a1;
                uz[p] = -2.0 * a2;
                al[p] = fma(a0, a0, fma(a1, a1, a2 * a2));
            }
#pragma unroll 1
            for (int j = 0; j < kChunk; ++j) {
                const int64_t tp = j0 + j;
                double acc = 0.0;
                if (tp < c1) {
                    const double* h = rec + tp * kRec;
#pragma unroll
                    for (int p = 0; p < 7; ++p) {
                        double sacc = 0.0;
#pragma unroll
                        for (int q = 0; q < 7; ++q) {
                            const double* rq = h + 5 * q;
                            const double s2 = fma(ux[p], rq[0], fma(uy[p], rq[1], fma(uz[p], rq[2], fma(al[p], rq[3], rq[4]))));
                            const double y = __builtin_amdgcn_rsq(s2);
                            sacc = fma(y, fma(-s2, y * y, 3.0), sacc);
                        }
                        acc = fma(pw[p], sacc, acc);
                    }
                }
                put(j, tp, acc * kInv4Pi);
            }
        } else {
            double px[7], py[7], pz[7];
#pragma unroll
            for (int p = 0; p < 7; ++p) {
                px[p] = g[3 * p];
                py[p] = g[3 * p + 1];
                pz[p] = g[3 * p + 2];
            }
#pragma unroll 1
            for (int j = 0; j < kChunk; ++j) {
                const int64_t tp = j0 + j;
                double acc = 0.0;
                if (tp < c1) {
                    const double* h = geo + tp * kGeo;
#pragma unroll
                    for (int q = 0; q < 7; ++q) {
                        const double yx = h[3 * q], yy = h[3 * q + 1], yz = h[3 * q + 2];
                        double sacc = 0.0;
#pragma unroll
                        for (int p = 0; p < 7; ++p) {
                            const double dx = px[p] - yx, dy = py[p] - yy, dz = pz[p] - yz;
                            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                            const double y = __builtin_amdgcn_rsq(r2);
                            sacc = fma(pw[p] * y, fma(-r2, y * y, 3.0), sacc);
                        }
                        acc = fma(h[21 + q], sacc, acc);
                    }
                }
                put(j, tp, acc * kInv4Pi);
            }
        }
        if (staged) {
            __builtin_amdgcn_wave_barrier();   // stage[wave] is private to this wave; order write -> read
            // lanes 8i .. 8i+7 write listed row (8 pass + i) of the tile, 16 bytes each
#pragma unroll
            for (int pass = 0; pass < 8; ++pass) {
                const int row = pass * 8 + (lane >> 3);
                const int col = (lane & 7) * 2;
                const double2 v = make_double2(stage[wave][row][col], stage[wave][row][col + 1]);
                *reinterpret_cast<double2*>(I + (int64_t(rb) * kTile + row) * ld + (j0 - col0) + col) = v;
            }
            __builtin_amdgcn_wave_barrier();   // reads done before the next chunk overwrites stage
        }
    }
}

__device__ __forceinline__ void load3(const double* __restrict__ V, int32_t i, double* o) {
    o[0] = V[3 * int64_t(i)];
    o[1] = V[3 * int64_t(i) + 1];
    o[2] = V[3 * int64_t(i) + 2];
}

__device__ __forceinline__ double inv_norm(double x, double y, double z) {
    return 1.0 / sqrt(x * x + y * y + z * z);
}

__device__ __forceinline__ double tri_area2(const double* a, const double* b, const double* c) {
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double x = u[1] * v[2] - u[2] * v[1], y = u[2] * v[0] - u[0] * v[2], z = u[0] * v[1] - u[1] * v[0];
    return 0.5 * sqrt(x * x + y * y + z * z);
}

// Same triangle.  z = x^ - y^ fills the hexagon with vertices +-(1,0), +-(1,1), +-(0,1); on each of
// its six triangles z = xi (v_i + eta (v_{i+1} - v_i)), and for fixed z the anchor y^ runs over a
// copy of the reference triangle scaled by (1 - xi).  With x - y = M z, M = [B-A, C-B], the
// integrand is (1-xi)^2 mu1 / |M (v_i + eta (v_{i+1}-v_i))|; xi and the anchor integrate to 1/6,
// and opposite hexagon triangles give equal values, leaving (1/3) sum_{i<3} int deta / |M w_i|.
__global__ void k_near_coincident(const double* __restrict__ V, const int32_t* __restrict__ vs,
                                  const int32_t* __restrict__ t1, int64_t n, int ng,
                                  const double* __restrict__ gx, const double* __restrict__ gw,
                                  double* __restrict__ I, int64_t ld, const int64_t* __restrict__ tgt) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double A[3], B[3], C[3];
    load3(V, vs[5 * i], A);
    load3(V, vs[5 * i + 1], B);
    load3(V, vs[5 * i + 2], C);
    double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double e2[3] = {C[0] - B[0], C[1] - B[1], C[2] - B[2]};
    const double hv[4][2] = {{1.0, 0.0}, {1.0, 1.0}, {0.0, 1.0}, {-1.0, 0.0}};
    double acc = 0.0;
    for (int s = 0; s < 3; ++s)
        for (int b = 0; b < ng; ++b) {
            double eta = gx[b];
            double w1 = hv[s][0] + eta * (hv[s + 1][0] - hv[s][0]);
            double w2 = hv[s][1] + eta * (hv[s + 1][1] - hv[s][1]);
            acc += gw[b] * inv_norm(w1 * e1[0] + w2 * e2[0], w1 * e1[1] + w2 * e2[1], w1 * e1[2] + w2 * e2[2]);
        }
    double ar = tri_area2(A, B, C);
    int64_t t = t1[i];
    const double val = acc * (1.0 / 3.0) * 4.0 * ar * ar * kInv4Pi;
    if (tgt) {
        if (tgt[2 * i] >= 0) I[tgt[2 * i]] = val;
    } else {
        I[t * ld + t] = val;
    }
}

// Common edge A-B: x - y = w1 (B-A) + w2 (C-B) - w3 (C'-B) with w = (s - s', t, t').  The cone
// {w2, w3 >= 0} is cut into four pieces on which max(w1,0) + max(w3, w2-w1) is linear; on each,
// w = xi b(eta) with b on the unit level set.  The anchor s' and xi integrate to 1/6, leaving
// (1/6) sum_R int int J_R(eta) / |D_R(eta)| d eta, J_R = 1 (square faces) or eta1 (triangular).
__global__ void k_near_edge(const double* __restrict__ V, const int32_t* __restrict__ vs,
                            const int32_t* __restrict__ t1, const int32_t* __restrict__ t2, int64_t n,
                            int ng, const double* __restrict__ gx, const double* __restrict__ gw,
                            double* __restrict__ I, int64_t ld, const int64_t* __restrict__ tgt) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double A[3], B[3], C[3], C2[3];
    load3(V, vs[5 * i], A);
    load3(V, vs[5 * i + 1], B);
    load3(V, vs[5 * i + 2], C);
    load3(V, vs[5 * i + 3], C2);
    double e1[3], e2[3], e3[3];
    for (int k = 0; k < 3; ++k) { e1[k] = B[k] - A[k]; e2[k] = C[k] - B[k]; e3[k] = C2[k] - B[k]; }
    double acc = 0.0;
    for (int b = 0; b < ng; ++b) {
        const double h1 = gx[b];
        for (int c = 0; c < ng; ++c) {
            const double h2 = gx[c];
            const double wbc = gw[b] * gw[c];
            // piece 1: b = (h1, h2, 1-h1), J = 1
            // piece 2: b = (h1 (1-h2), 1, h1 h2), J = h1
            // piece 3: b = (-h1 (1-h2), h1 h2, 1), J = h1
            // piece 4: b = (-h1, 1-h1, h2), J = 1
            const double bb[4][3] = {{h1, h2, 1.0 - h1},
                                     {h1 * (1.0 - h2), 1.0, h1 * h2},
                                     {-h1 * (1.0 - h2), h1 * h2, 1.0},
                                     {-h1, 1.0 - h1, h2}};
            const double jac[4] = {1.0, h1, h1, 1.0};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double dx = bb[r][0] * e1[0] + bb[r][1] * e2[0] - bb[r][2] * e3[0];
                double dy = bb[r][0] * e1[1] + bb[r][1] * e2[1] - bb[r][2] * e3[1];
                double dz = bb[r][0] * e1[2] + bb[r][1] * e2[2] - bb[r][2] * e3[2];
                acc += wbc * jac[r] * inv_norm(dx, dy, dz);
            }
        }
    }
    double val = acc * (1.0 / 6.0) * 4.0 * tri_area2(A, B, C) * tri_area2(A, B, C2) * kInv4Pi;
    int64_t a = t1[i], b = t2[i];
    if (tgt) {   // panel of the pair matrix: the positions this pair has in it (-1: outside)
        if (tgt[2 * i] >= 0) I[tgt[2 * i]] = val;
        if (tgt[2 * i + 1] >= 0) I[tgt[2 * i + 1]] = val;
    } else {
        I[a * ld + b] = val;
        I[b * ld + a] = val;
    }
}

// Common vertex A: x^ = xi (1, eta1), y^ = xi (eta2, eta2 eta3) on {s' <= s} and the mirror piece;
// Jacobian xi^3 eta2, the xi integral of xi^2 is 1/3.
__global__ void k_near_vertex(const double* __restrict__ V, const int32_t* __restrict__ vs,
                              const int32_t* __restrict__ t1, const int32_t* __restrict__ t2, int64_t n,
                              int ng, const double* __restrict__ gx, const double* __restrict__ gw,
                              double* __restrict__ I, int64_t ld, const int64_t* __restrict__ tgt) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double A[3], B[3], C[3], B2[3], C2[3];
    load3(V, vs[5 * i], A);
    load3(V, vs[5 * i + 1], B);
    load3(V, vs[5 * i + 2], C);
    load3(V, vs[5 * i + 3], B2);
    load3(V, vs[5 * i + 4], C2);
    double f1[3], f2[3], g1[3], g2[3];
    for (int k = 0; k < 3; ++k) { f1[k] = B[k] - A[k]; f2[k] = C[k] - B[k]; g1[k] = B2[k] - A[k]; g2[k] = C2[k] - B2[k]; }
    double acc = 0.0;
    for (int b = 0; b < ng; ++b) {
        const double h1 = gx[b];
        // P = (1, h1) on both charts
        double MP[3], NP[3];
        for (int k = 0; k < 3; ++k) { MP[k] = f1[k] + h1 * f2[k]; NP[k] = g1[k] + h1 * g2[k]; }
        for (int c = 0; c < ng; ++c) {
            const double h2 = gx[c];
            for (int d = 0; d < ng; ++d) {
                const double h3 = gx[d];
                const double q0 = h2, q1 = h2 * h3;
                double MQ[3], NQ[3];
                for (int k = 0; k < 3; ++k) { MQ[k] = q0 * f1[k] + q1 * f2[k]; NQ[k] = q0 * g1[k] + q1 * g2[k]; }
                double s = inv_norm(MP[0] - NQ[0], MP[1] - NQ[1], MP[2] - NQ[2]) +
                           inv_norm(MQ[0] - NP[0], MQ[1] - NP[1], MQ[2] - NP[2]);
                acc += gw[b] * gw[c] * gw[d] * h2 * s;
            }
        }
    }
    double val = acc * (1.0 / 3.0) * 4.0 * tri_area2(A, B, C) * tri_area2(A, B2, C2) * kInv4Pi;
    int64_t a = t1[i], b = t2[i];
    if (tgt) {   // panel of the pair matrix: the positions this pair has in it (-1: outside)
        if (tgt[2 * i] >= 0) I[tgt[2 * i]] = val;
        if (tgt[2 * i + 1] >= 0) I[tgt[2 * i + 1]] = val;
    } else {
        I[a * ld + b] = val;
        I[b * ld + a] = val;
    }
}

// W over 64 x 64 dof tiles above the diagonal.  Wave w of the block takes rows d0 + 16w .. +15 one
// at a time; lane l takes column e = e0 + l.  The row dof's star (triangle T_i, J_i) is
// wave-uniform and comes through scalar loads; each lane keeps its column dof's star (T'_k, J_k) in
// registers.  For a row, all of its I(T_i, T'_k) loads (up to kReg x kReg, neighbouring columns of
// a few rows of I) are issued before any is consumed, so a wave keeps dozens of loads in flight;
// stars longer than kReg (junction dofs) finish in a slower loop.  Each W entry is computed once
// and written to both halves (exactly symmetric); the mirrored tile is transposed through LDS so
// both writes are coalesced.
constexpr int kCT = 64;    // tile edge (dofs)
constexpr int kReg = 6;    // star entries handled in the unrolled path (a flat interior star has 6)

__global__ __launch_bounds__(256) void k_contract(const double* __restrict__ I, int64_t ldI, const int32_t* __restrict__ rowmap,
                                                  int64_t col0, int64_t N,
                                                  const int64_t* __restrict__ dof_ptr, const int32_t* __restrict__ dof_tri,
                                                  const double* __restrict__ dof_J, const int2* __restrict__ tiles,
                                                  int64_t ntiles, double* __restrict__ W, float* __restrict__ W32,
                                                  int64_t ldw) {
    __shared__ double tileT[kCT][kCT + 1];
    // blocks of one XCD (blockIdx % 8) walk a contiguous run of tiles, so neighbouring tiles that
    // re-read the same rows of I meet in that XCD's L2
    const int64_t per = (ntiles + 7) / 8;
    const int64_t t = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntiles) return;
    const int2 tl = tiles[t];
    const int bd = tl.x, be = tl.y;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t e = int64_t(be) * kCT + lane;
    const bool ev = e < N;
    const int64_t kb = ev ? dof_ptr[e] : 0;
    const int ne = ev ? int(dof_ptr[e + 1] - kb) : 0;
    int Tk[kReg];
    double Jx[kReg], Jy[kReg], Jz[kReg];
#pragma unroll
    for (int k = 0; k < kReg; ++k) {
        const bool h = k < ne;
        Tk[k] = h ? dof_tri[kb + k] - int32_t(col0) : 0;   // column within I (>= 0 by the choice of col0)
        Jx[k] = h ? dof_J[3 * (kb + k)] : 0.0;
        Jy[k] = h ? dof_J[3 * (kb + k) + 1] : 0.0;
        Jz[k] = h ? dof_J[3 * (kb + k) + 2] : 0.0;
    }
    for (int r = 0; r < 16; ++r) {
        const int64_t d = int64_t(bd) * kCT + wave * 16 + r;
        double acc = 0.0;
        if (d < N) {
            const int64_t i0 = dof_ptr[d];
            const int ni = int(dof_ptr[d + 1] - i0);
            const double* Ir[kReg];
            double ja[kReg], jb[kReg], jc[kReg];
#pragma unroll
            for (int i = 0; i < kReg; ++i) {
                const bool h = i < ni;
                const int32_t T = h ? dof_tri[i0 + i] : -1;
                Ir[i] = I + int64_t(T < 0 ? 0 : (rowmap ? rowmap[T] : T)) * ldI;
                ja[i] = h ? dof_J[3 * (i0 + i)] : 0.0;
                jb[i] = h ? dof_J[3 * (i0 + i) + 1] : 0.0;
                jc[i] = h ? dof_J[3 * (i0 + i) + 2] : 0.0;
            }
            double v[kReg][kReg];
#pragma unroll
            for (int i = 0; i < kReg; ++i)
#pragma unroll
                for (int k = 0; k < kReg; ++k) v[i][k] = (i < ni && k < ne) ? Ir[i][Tk[k]] : 0.0;
#pragma unroll
            for (int i = 0; i < kReg; ++i)
#pragma unroll
                for (int k = 0; k < kReg; ++k) acc = fma(v[i][k], ja[i] * Jx[k] + jb[i] * Jy[k] + jc[i] * Jz[k], acc);
            // junction stars: the entries beyond the unrolled ones
            if (ni > kReg || ne > kReg) {
                for (int i = 0; i < ni; ++i) {
                    const int64_t qi = i0 + i;
                    const int32_t T = dof_tri[qi];
                    const double* Irow = I + int64_t(rowmap ? rowmap[T] : T) * ldI - col0;
                    const double j0 = dof_J[3 * qi], j1 = dof_J[3 * qi + 1], j2 = dof_J[3 * qi + 2];
                    for (int k = (i < kReg ? kReg : 0); k < ne; ++k) {
                        const int64_t q = kb + k;
                        acc = fma(Irow[dof_tri[q]], j0 * dof_J[3 * q] + j1 * dof_J[3 * q + 1] + j2 * dof_J[3 * q + 2], acc);
                    }
                }
            }
            if (bd != be || e >= d) {   // columns past N: zero padding
                W[d * ldw + e] = acc;
                if (W32) W32[d * ldw + e] = float(acc);
            }
        }
        tileT[wave * 16 + r][lane] = acc;
    }
    __syncthreads();
    // mirrored half: W[e'][d'] = entry (d', e') for the tile's rows d' and columns e'
    for (int q = threadIdx.x; q < kCT * kCT; q += 256) {
        const int re = q / kCT, cd = q % kCT;
        const int64_t em = int64_t(be) * kCT + re, dm = int64_t(bd) * kCT + cd;
        if (em < N && dm < N && (bd != be || dm < em)) {
            W[em * ldw + dm] = tileT[cd][re];
            if (W32) W32[em * ldw + dm] = float(tileT[cd][re]);
        }
    }
}

// Staged form of the same contraction, for column blocks whose stars together hold at most kCap
// triangles.  With y_T(e) = sum over the star of e of J(T',e) I(T,T'), an entry is
// W(d,e) = sum over T in the star of d of J(T,d) . y_T(e).  The 64 columns of a tile share one
// sorted list C of the triangles in their stars (at most kCap), and each lane holds the first kRegC
// entries of its column's star as positions in C (longer junction stars finish from memory).  Wave
// w of the block owns 16 rows; it walks the triangles T of their stars (one group per triangle,
// prepared on the host), loads I(T, C) once with neighbouring lanes on neighbouring list entries,
// stages it in LDS, forms y_T for all 64 columns from LDS and adds J(T,d) . y_T into the rows d
// whose star holds T.  Accumulators live in LDS, which then feeds both the direct and the mirrored
// (transposed) coalesced write.  Columns past N (the padding of W) are written as zero.
constexpr int kRegC = 8;
constexpr int kCap = kCT * kRegC;

// One wave's walk over its groups for a column list of NCH chunks of 64 entries.  The segment
// I(T, C) of a group is loaded two groups ahead, every chunk of it unconditionally (lanes past the
// list repeat its last entry, and the two loads past the last group repeat that group), so each
// wait for a segment leaves the younger segment's loads in flight.  An odd group count ends with a
// step that stages a segment and adds nothing.
template <int NCH>
__device__ __forceinline__ void contract_walk(
    const double* __restrict__ I, int64_t ldI, const int32_t* __restrict__ rowmap, const int32_t* __restrict__ ctri,
    int nc, int64_t col0, const int4* __restrict__ rg, const int2* __restrict__ rg_ent, int g0, int g1,
    const double* __restrict__ dof_J, const int32_t* __restrict__ col_loc, int64_t kb, int ne, const int (&loc)[kRegC],
    const double (&Jx)[kRegC], const double (&Jy)[kRegC], const double (&Jz)[kRegC], double* __restrict__ sw,
    double* __restrict__ arow, int lane) {
    if (g0 >= g1) return;
    int cidx[NCH];
#pragma unroll
    for (int m = 0; m < NCH; ++m) cidx[m] = ctri[min(m * kCT + lane, nc - 1)] - int32_t(col0);
    double A[NCH], B[NCH];
    auto fetch = [&](double (&dst)[NCH], int g) {
        const int T = rg[min(g, g1 - 1)].x;
        const double* row = I + int64_t(rowmap ? rowmap[T] : T) * ldI;
#pragma unroll
        for (int m = 0; m < NCH; ++m) dst[m] = row[cidx[m]];
    };
    auto step = [&](double (&cur)[NCH], int g) {
        const int4 G = rg[min(g, g1 - 1)];   // (triangle, rows, first entry, -)
        const int ny = g < g1 ? G.y : 0;
#pragma unroll
        for (int m = 0; m < NCH; ++m) sw[m * kCT + lane] = cur[m];
        fetch(cur, g + 2);
        __builtin_amdgcn_wave_barrier();   // sw belongs to this wave: order write -> read
        double yx = 0.0, yy = 0.0, yz = 0.0;
#pragma unroll
        for (int k = 0; k < kRegC; ++k) {
            const double v = sw[loc[k]];
            yx = fma(Jx[k], v, yx);
            yy = fma(Jy[k], v, yy);
            yz = fma(Jz[k], v, yz);
        }
        if (ne > kRegC) {   // junction columns: star entries past the registers, from memory
            for (int k = kRegC; k < ne; ++k) {
                const int64_t q = kb + k;
                const double v = sw[col_loc[q]];
                yx = fma(dof_J[3 * q], v, yx);
                yy = fma(dof_J[3 * q + 1], v, yy);
                yz = fma(dof_J[3 * q + 2], v, yz);
            }
        }
        for (int i = 0; i < ny; ++i) {
            const int2 en = rg_ent[G.z + i];   // (row in the wave's 16, star entry of that row)
            const double* j = dof_J + 3 * int64_t(en.y);
            double& a = arow[en.x * (kCT + 1) + lane];
            a = fma(j[0], yx, fma(j[1], yy, fma(j[2], yz, a)));
        }
        __builtin_amdgcn_wave_barrier();   // reads of sw done before the next step overwrites it
    };
    fetch(A, g0);
    fetch(B, g0 + 1);
    for (int g = g0; g < g1; g += 2) {
        step(A, g);
        step(B, g + 1);
    }
}

__global__ __launch_bounds__(256, 3) void k_contract_staged(
    const double* __restrict__ I, int64_t ldI, const int32_t* __restrict__ rowmap, int64_t col0, int64_t N,
    const int32_t* __restrict__ cb_ptr,
    const int32_t* __restrict__ cb_tri, const int64_t* __restrict__ dof_ptr, const int32_t* __restrict__ col_loc,
    const double* __restrict__ dof_J, const int32_t* __restrict__ rg_ptr, const int4* __restrict__ rg,
    const int2* __restrict__ rg_ent, const int2* __restrict__ tiles, int64_t ntiles, double* __restrict__ W,
    float* __restrict__ W32, int64_t ldw) {
    __shared__ double acc[kCT][kCT + 1];
    __shared__ double seg[4][kCap];
    const int64_t per = (ntiles + 7) / 8;
    const int64_t t = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntiles) return;
    const int2 tl = tiles[t];
    const int bd = __builtin_amdgcn_readfirstlane(tl.x), be = __builtin_amdgcn_readfirstlane(tl.y);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t e = int64_t(be) * kCT + lane;
    const bool ev = e < N;
    const int64_t kb = ev ? dof_ptr[e] : 0;
    const int ne = ev ? int(dof_ptr[e + 1] - kb) : 0;
    int loc[kRegC];
    double Jx[kRegC], Jy[kRegC], Jz[kRegC];
    // unconditional loads of in-range entries (entries past the star repeat its last one, or entry
    // 0 for a padding column), masked afterwards: all of them are in flight together
    const int64_t klast = ne > 0 ? kb + ne - 1 : 0;
#pragma unroll
    for (int k = 0; k < kRegC; ++k) {
        const int64_t q = min<int64_t>(kb + k, klast);
        loc[k] = col_loc[q];
        Jx[k] = dof_J[3 * q];
        Jy[k] = dof_J[3 * q + 1];
        Jz[k] = dof_J[3 * q + 2];
    }
#pragma unroll
    for (int k = 0; k < kRegC; ++k)
        if (k >= ne) {
            loc[k] = 0;
            Jx[k] = Jy[k] = Jz[k] = 0.0;
        }
    const int c0 = cb_ptr[be];
    const int nc = cb_ptr[be + 1] - c0;
    double* arow = &acc[wave * 16][0];
#pragma unroll
    for (int r = 0; r < 16; ++r) arow[r * (kCT + 1) + lane] = 0.0;
    const int rb = bd * 4 + wave;
    const int g0 = rg_ptr[rb], g1 = rg_ptr[rb + 1];
    switch ((nc + kCT - 1) / kCT) {
#define BEM_WALK(n)                                                                                                   \
    case n:                                                                                                           \
        contract_walk<n>(I, ldI, rowmap, cb_tri + c0, nc, col0, rg, rg_ent, g0, g1, dof_J,  col_loc, kb, ne, loc, Jx, \
                         Jy, Jz, seg[wave], arow, lane);                                                              \
        break;
        BEM_WALK(1) BEM_WALK(2) BEM_WALK(3) BEM_WALK(4) BEM_WALK(5) BEM_WALK(6) BEM_WALK(7) BEM_WALK(8)
#undef BEM_WALK
        default: break;   // the host sends longer lists to the general kernel
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t d = int64_t(bd) * kCT + wave * 16 + r;
        if (d < N && (bd != be || e >= d)) {
            const double v = arow[r * (kCT + 1) + lane];
            W[d * ldw + e] = v;
            if (W32) W32[d * ldw + e] = float(v);
        }
    }
    for (int q = threadIdx.x; q < kCT * kCT; q += 256) {
        const int re = q / kCT, cd = q % kCT;
        const int64_t em = int64_t(be) * kCT + re, dm = int64_t(bd) * kCT + cd;
        if (em < N && dm < N && (bd != be || dm < em)) {
            const double v = acc[cd][re];
            W[em * ldw + dm] = v;
            if (W32) W32[em * ldw + dm] = float(v);
        }
    }
}

// L[k][d] = -sum over the star of d of c (g_k . n_T) |T| / 3
__global__ void k_rhs(const int64_t* __restrict__ dof_ptr, const int32_t* __restrict__ dof_tri,
                      const int8_t* __restrict__ dof_c, const double* __restrict__ normal,
                      const double* __restrict__ area, int64_t N, const double* __restrict__ g, int k,
                      double* __restrict__ L) {
    int64_t d = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (d >= N) return;
    for (int c = 0; c < k; ++c) {
        double s = 0.0;
        for (int64_t e = dof_ptr[d]; e < dof_ptr[d + 1]; ++e) {
            int64_t t = dof_tri[e];
            double gn = g[3 * c] * normal[3 * t] + g[3 * c + 1] * normal[3 * t + 1] + g[3 * c + 2] * normal[3 * t + 2];
            s -= double(dof_c[e]) * gn * area[t] * (1.0 / 3.0);
        }
        L[int64_t(c) * N + d] = s;
    }
}

// per element (triangle: 3 corners, segment: 2 ends) the jump of sum_d phi_d psi_d at its corners
__global__ void k_jump_values(const int64_t* __restrict__ tri_ptr, const int32_t* __restrict__ tri_dof,
                              const int8_t* __restrict__ tri_corner, const int8_t* __restrict__ tri_c,
                              int64_t nt, int corners, const double* __restrict__ phi, double* __restrict__ out) {
    int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    double j[3] = {0.0, 0.0, 0.0};
    for (int64_t e = tri_ptr[t]; e < tri_ptr[t + 1]; ++e) j[tri_corner[e]] += double(tri_c[e]) * phi[tri_dof[e]];
    for (int a = 0; a < corners; ++a) out[corners * t + a] = j[a];
}

// two-dimensional right-hand side: L[k][d] = -sum over the star of d of c (g_k . n_s) |s| / 2
__global__ void k_rhs2d(const int64_t* __restrict__ dof_ptr, const int32_t* __restrict__ dof_seg,
                        const int8_t* __restrict__ dof_c, const double* __restrict__ normal,
                        const double* __restrict__ length, int64_t N, const double* __restrict__ g, int k,
                        double* __restrict__ L) {
    int64_t d = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (d >= N) return;
    for (int c = 0; c < k; ++c) {
        double s = 0.0;
        for (int64_t e = dof_ptr[d]; e < dof_ptr[d + 1]; ++e) {
            const int64_t t = dof_seg[e];
            const double gn = g[3 * c] * normal[3 * t] + g[3 * c + 1] * normal[3 * t + 1];
            s -= double(dof_c[e]) * gn * length[t] * 0.5;
        }
        L[int64_t(c) * N + d] = s;
    }
}

inline unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }

// Brackets device work on a stream with two events; the elapsed time is read once the work is done,
// so timing never stalls the host in the middle of the pipeline.
struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit EventTimer(hipStream_t st) : s(st) {
        HIP_CHECK(hipEventCreate(&a));
        HIP_CHECK(hipEventCreate(&b));
        HIP_CHECK(hipEventRecord(a, s));
    }
    void stop() { HIP_CHECK(hipEventRecord(b, s)); }
    double seconds() {
        HIP_CHECK(hipEventSynchronize(b));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, a, b));
        return ms * 1e-3;
    }
    EventTimer(const EventTimer&) = delete;
    EventTimer& operator=(const EventTimer&) = delete;
    ~EventTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Host side of the staged contraction.  Column blocks are 64 consecutive dofs: the sorted union
// of their stars' triangles and, per star entry, its position in that union.  Row blocks are 16
// consecutive dofs: one group per triangle of their stars, listing the (row, star entry) pairs
// that hold it.  Tiles whose column block's union exceeds kCap triangles take the general kernel.
struct ContractPlan {
    std::vector<int32_t> cb_ptr, cb_tri, col_loc, rg_ptr;
    std::vector<int4> rg;
    std::vector<int2> rg_ent, fast, slow;
};

ContractPlan contract_plan(const MeshTopo& m) {
    const int64_t N = m.N;
    const int64_t ncb = (N + kCT - 1) / kCT, nrb = ncb * 4;
    const int64_t nnz = m.dof_ptr[N];
    if (nnz > INT32_MAX) fail(BEM_E_UNSUPPORTED, "more than 2^31 star entries");
    ContractPlan P;
    P.col_loc.assign(size_t(nnz), 0);
    P.cb_ptr.assign(size_t(ncb) + 1, 0);
    std::vector<uint8_t> ok(static_cast<size_t>(ncb), 1);
    std::vector<std::vector<int32_t>> lists(static_cast<size_t>(ncb));
    parallel_for(ncb, [&](int64_t lo, int64_t hi) {
        for (int64_t b = lo; b < hi; ++b) {
            const int64_t e0 = b * kCT, e1 = std::min<int64_t>(N, e0 + kCT);
            std::vector<int32_t>& L = lists[size_t(b)];
            for (int64_t e = e0; e < e1; ++e) {
                for (int64_t q = m.dof_ptr[e]; q < m.dof_ptr[e + 1]; ++q) L.push_back(m.dof_tri[q]);
            }
            std::sort(L.begin(), L.end());
            L.erase(std::unique(L.begin(), L.end()), L.end());
            if (int64_t(L.size()) > kCap) ok[size_t(b)] = 0;
            for (int64_t q = m.dof_ptr[e0]; q < m.dof_ptr[e1]; ++q)
                P.col_loc[size_t(q)] = int32_t(std::lower_bound(L.begin(), L.end(), m.dof_tri[q]) - L.begin());
        }
    }, 8);
    for (int64_t b = 0; b < ncb; ++b) P.cb_ptr[size_t(b) + 1] = P.cb_ptr[size_t(b)] + int32_t(lists[size_t(b)].size());
    P.cb_tri.reserve(size_t(P.cb_ptr.back()));
    for (auto& L : lists) P.cb_tri.insert(P.cb_tri.end(), L.begin(), L.end());

    // row groups: (triangle, row, entry) sorted by triangle then row
    std::vector<std::vector<int4>> groups(static_cast<size_t>(nrb));
    std::vector<std::vector<int2>> ents(static_cast<size_t>(nrb));
    parallel_for(nrb, [&](int64_t lo, int64_t hi) {
        std::vector<int4> key;   // (triangle, row, entry, -)
        for (int64_t b = lo; b < hi; ++b) {
            key.clear();
            for (int r = 0; r < 16; ++r) {
                const int64_t d = b * 16 + r;
                if (d >= N) break;
                for (int64_t q = m.dof_ptr[d]; q < m.dof_ptr[d + 1]; ++q) key.push_back(make_int4(m.dof_tri[q], r, int(q), 0));
            }
            std::sort(key.begin(), key.end(), [](const int4& a, const int4& c) { return a.x != c.x ? a.x < c.x : a.y < c.y; });
            std::vector<int4>& G = groups[size_t(b)];
            std::vector<int2>& E = ents[size_t(b)];
            for (size_t i = 0; i < key.size();) {
                size_t j = i;
                while (j < key.size() && key[j].x == key[i].x) ++j;
                G.push_back(make_int4(key[i].x, int(j - i), int(E.size()), 0));
                for (size_t k = i; k < j; ++k) E.push_back(make_int2(key[k].y, key[k].z));
                i = j;
            }
        }
    }, 32);
    P.rg_ptr.assign(size_t(nrb) + 1, 0);
    for (int64_t b = 0; b < nrb; ++b) P.rg_ptr[size_t(b) + 1] = P.rg_ptr[size_t(b)] + int32_t(groups[size_t(b)].size());
    P.rg.reserve(size_t(P.rg_ptr.back()));
    for (int64_t b = 0; b < nrb; ++b) {
        const int32_t base = int32_t(P.rg_ent.size());
        for (int4 g : groups[size_t(b)]) P.rg.push_back(make_int4(g.x, g.y, g.z + base, 0));
        P.rg_ent.insert(P.rg_ent.end(), ents[size_t(b)].begin(), ents[size_t(b)].end());
    }
    for (int64_t gd = 0; gd < ncb; ++gd)
        for (int64_t ge = gd; ge < ncb; ++ge) (ok[size_t(ge)] ? P.fast : P.slow).push_back(make_int2(int(gd), int(ge)));
    return P;
}

// ---- panel-by-panel assembly -------------------------------------------------------------------
// For meshes whose N_T x N_T pair matrix does not fit next to W: the dof row blocks (64 dofs) are
// grouped into panels whose rows number at most maxrows.  The rows of a panel are the triangles at
// the vertices of its blocks' dofs (the stars of those dofs, plus the few triangles at such a vertex
// whose jump coefficients there all vanish).  A panel computes I_P = I(R, [tmin, N_T)) for
// its rows R, each 64-row tile from the first column a tile (bd, be >= bd) of the panel can read
// it at, the near pairs that fall in it, and then contracts its tiles of the upper half of W (the
// mirrored writes fill the lower half).  Far work is about half of N_T^2 pairs in total, as in the
// one-shot path.  The layout needs only the number of dofs of each vertex, which forecast_dofs
// gets from counts: the first panel's far pass is queued before the host's sector analysis and
// runs while the host analyses the mesh, and the host filters each panel's near pairs while that
// panel's far pass runs.

// Dofs of each vertex before the sector analysis (Section 4.2: q_v sectors, q_v - 1 dofs).  Near a
// vertex v of a conforming multiscreen without point contacts, the triangles and edges at v cut a
// small sphere about v along a connected graph (one node per edge at v, one arc per triangle at v)
// whose faces are the sectors at v; Euler's formula gives q_v = T_v - E_v + 2 from the numbers T_v
// of triangles and E_v of edges at v.  The analysis confirms the forecast for every mesh it accepts;
// the caller compares the two before anything depends on the difference.
struct DofForecast {
    std::vector<int64_t> vt_ptr;      // triangles at each vertex (ascending), CSR over vertices
    std::vector<int32_t> vt;
    std::vector<int64_t> first_dof;   // nv + 1: dofs of vertex v are first_dof[v] .. first_dof[v + 1] - 1
    int64_t N = 0;
};

DofForecast forecast_dofs(const int32_t* T, int64_t nv, int64_t nt) {
    DofForecast f;
    f.vt_ptr.assign(static_cast<size_t>(nv) + 1, 0);
    for (int64_t i = 0; i < 3 * nt; ++i) ++f.vt_ptr[size_t(T[i]) + 1];
    for (int64_t v = 0; v < nv; ++v) f.vt_ptr[size_t(v) + 1] += f.vt_ptr[size_t(v)];
    f.vt.resize(static_cast<size_t>(3 * nt));
    {
        std::vector<int64_t> pos(f.vt_ptr.begin(), f.vt_ptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int a = 0; a < 3; ++a) f.vt[size_t(pos[size_t(T[3 * t + a])]++)] = int32_t(t);
    }
    std::vector<int64_t> nd(static_cast<size_t>(nv), 0);
    parallel_for(nv, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> nb;
        for (int64_t v = lo; v < hi; ++v) {
            const int64_t tv = f.vt_ptr[size_t(v) + 1] - f.vt_ptr[size_t(v)];
            if (tv == 0) continue;
            nb.clear();
            for (int64_t k = f.vt_ptr[size_t(v)]; k < f.vt_ptr[size_t(v) + 1]; ++k) {
                const int32_t* c = T + 3 * int64_t(f.vt[size_t(k)]);
                for (int a = 0; a < 3; ++a)
                    if (c[a] != v) nb.push_back(c[a]);
            }
            std::sort(nb.begin(), nb.end());
            const int64_t ev = std::unique(nb.begin(), nb.end()) - nb.begin();
            nd[size_t(v)] = std::max<int64_t>(0, tv - ev + 1);   // q_v - 1
        }
    }, 4096);
    f.first_dof.assign(static_cast<size_t>(nv) + 1, 0);
    for (int64_t v = 0; v < nv; ++v) f.first_dof[size_t(v) + 1] = f.first_dof[size_t(v)] + nd[size_t(v)];
    f.N = f.first_dof[size_t(nv)];
    return f;
}

// Panels of a dof numbering (first_dof, N dofs): consecutive row blocks whose rows (the triangles
// at the vertices of the blocks' dofs) number at most maxrows, each panel's first column, and the
// first column each row is read at.
struct PanelLayout {
    std::vector<int64_t> starts;                  // first row block of each panel, then the block count
    std::vector<int64_t> tmin;                    // each panel's first column (a multiple of 16)
    std::vector<std::vector<int32_t>> rows;       // each panel's row triangles, ascending
    std::vector<std::vector<int32_t>> rowfirst;   // per row: the first column a tile of the panel reads it at
    int64_t max_elems = 1;                        // entries of the largest panel
};

PanelLayout layout_panels(const std::vector<int64_t>& first_dof, int64_t N, const DofForecast& f, int64_t nt,
                          int64_t maxrows) {
    PanelLayout L;
    const int64_t nv = int64_t(first_dof.size()) - 1;
    const int64_t ncb = (N + kCT - 1) / kCT;
    // the vertices of each block's dofs, and the first column (a multiple of 16) that a tile
    // (bd, be >= bd) can read: every triangle of such a column block lies at a vertex with dofs
    // from the first dof of bd on
    auto vertex_of = [&](int64_t d) {
        return int64_t(std::upper_bound(first_dof.begin(), first_dof.end(), d) - first_dof.begin()) - 1;
    };
    std::vector<int64_t> vlo(static_cast<size_t>(ncb)), vhi(static_cast<size_t>(ncb)), col(static_cast<size_t>(ncb));
    std::vector<int64_t> sm(static_cast<size_t>(nv) + 1, nt);
    for (int64_t v = nv - 1; v >= 0; --v) {
        const bool has = first_dof[size_t(v) + 1] > first_dof[size_t(v)] && f.vt_ptr[size_t(v) + 1] > f.vt_ptr[size_t(v)];
        sm[size_t(v)] = std::min<int64_t>(sm[size_t(v) + 1], has ? f.vt[size_t(f.vt_ptr[size_t(v)])] : nt);
    }
    for (int64_t b = 0; b < ncb; ++b) {
        vlo[size_t(b)] = vertex_of(b * kCT);
        vhi[size_t(b)] = vertex_of(std::min<int64_t>(N, b * kCT + kCT) - 1);
        col[size_t(b)] = sm[size_t(vlo[size_t(b)])] / kGrp * kGrp;
    }
    std::vector<int32_t> stamp(static_cast<size_t>(nt), -1), first_block(static_cast<size_t>(nt), 0);
    int64_t b0 = 0;
    int id = 0;
    while (b0 < ncb) {
        std::vector<int32_t> rows, add;
        int64_t b1 = b0;
        while (b1 < ncb) {
            add.clear();
            for (int64_t v = vlo[size_t(b1)]; v <= vhi[size_t(b1)]; ++v) {
                if (first_dof[size_t(v) + 1] == first_dof[size_t(v)]) continue;
                for (int64_t k = f.vt_ptr[size_t(v)]; k < f.vt_ptr[size_t(v) + 1]; ++k) {
                    const int32_t T = f.vt[size_t(k)];
                    if (stamp[size_t(T)] != id) {
                        stamp[size_t(T)] = id;
                        first_block[size_t(T)] = int32_t(b1);
                        add.push_back(T);
                    }
                }
            }
            if (b1 > b0 && int64_t(rows.size() + add.size()) > maxrows) {
                for (int32_t T : add) stamp[size_t(T)] = -1;
                break;
            }
            rows.insert(rows.end(), add.begin(), add.end());
            ++b1;
        }
        // ascending order: the stamped triangles between the smallest and the largest row
        if (!rows.empty()) {
            const int32_t lo = *std::min_element(rows.begin(), rows.end()), hi = *std::max_element(rows.begin(), rows.end());
            size_t n = 0;
            for (int32_t T = lo; T <= hi; ++T)
                if (stamp[size_t(T)] == id) rows[n++] = T;
        }
        std::vector<int32_t> firsts(rows.size());
        for (size_t i = 0; i < rows.size(); ++i) firsts[i] = int32_t(col[size_t(first_block[size_t(rows[i])])]);
        const int64_t tmin = col[size_t(b0)];
        L.max_elems = std::max<int64_t>(L.max_elems, int64_t(rows.size()) * ((nt - tmin + 7) / 8 * 8));
        L.starts.push_back(b0);
        L.tmin.push_back(tmin);
        L.rows.push_back(std::move(rows));
        L.rowfirst.push_back(std::move(firsts));
        b0 = b1;
        ++id;
    }
    L.starts.push_back(ncb);
    return L;
}

// Far-pass tiles of a panel.  Row tile rb takes the column tiles cstart[rb] .. nct - 1.  The row
// tiles go in groups of kRowGroup, and a group lists its tiles column by column (row tiles in order
// within a column), at positions gptr[g] .. gptr[g + 1] - 1.  The four waves of a workgroup then
// read the same column records, and so do the workgroups next to it, which the dispatcher deals
// round-robin to the XCDs: a column tile's records come from HBM about once per group and XCD
// instead of once per row tile.  Column c's first position in its group is the number of the
// group's tiles left of it, the sum over the group's row tiles of max(0, c - cstart[rb]).
// Grid: (groups, column tiles / 256), one thread per column tile.
constexpr int kRowGroup = 64;
__global__ __launch_bounds__(256) void k_rect_tiles(const int32_t* __restrict__ cstart, const int64_t* __restrict__ gptr,
                                                    int32_t nrt, int32_t nct, int2* __restrict__ out) {
    __shared__ int32_t cs[kRowGroup];
    const int g = int(blockIdx.x);
    const int rb0 = g * kRowGroup, nr = min(kRowGroup, nrt - rb0);
    if (int(threadIdx.x) < nr) cs[threadIdx.x] = cstart[rb0 + int(threadIdx.x)];
    __syncthreads();
    const int c = int(blockIdx.y) * int(blockDim.x) + int(threadIdx.x);
    if (c >= nct) return;
    int64_t pos = gptr[g];
    for (int i = 0; i < nr; ++i) pos += max(0, c - cs[i]);
    for (int i = 0; i < nr; ++i)
        if (cs[i] <= c) out[pos++] = make_int2(rb0 + i, c);
}

// A second stream for host-to-device copies, so that they run beside the kernels queued on the
// first: each buffer belongs to the first stream (it is released in that stream's order), and the
// first stream waits for its copy before anything queued on it later, so no kernel reads it early and
// no release (an exception's included) precedes the copy.
struct SideCopies {
    bem_ctx* ctx;
    hipStream_t main, side = nullptr;
    hipEvent_t done = nullptr;
    SideCopies(bem_ctx* c, hipStream_t s) : ctx(c), main(s) {
        side = acquire_stream(c);
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            release_stream(c, side);
            fail(BEM_E_DEVICE, "hipEventCreateWithFlags failed");
        }
    }
    template <class T>
    DeviceBuffer upload(const std::vector<T>& v) {
        DeviceBuffer b(std::max<size_t>(1, v.size()) * sizeof(T), main);
        if (!v.empty()) {
            HIP_CHECK(hipMemcpyAsync(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, side));
            HIP_CHECK(hipEventRecord(done, side));
            HIP_CHECK(hipStreamWaitEvent(main, done, 0));
        }
        return b;
    }
    SideCopies(const SideCopies&) = delete;
    SideCopies& operator=(const SideCopies&) = delete;
    ~SideCopies() {
        (void)hipStreamSynchronize(side);   // its copies wait for no kernel: back to the list idle
        if (done) (void)hipEventDestroy(done);
        release_stream(ctx, side);
    }
};

// Device copies of the contraction plan, shared by all panels
struct PlanDevice {
    DeviceBuffer cb_ptr, cb_tri, col_loc, rg_ptr, rg, rg_ent, fast, slow;
    explicit PlanDevice(const ContractPlan& plan, SideCopies& up)
        : cb_ptr(up.upload(plan.cb_ptr)), cb_tri(up.upload(plan.cb_tri)), col_loc(up.upload(plan.col_loc)),
          rg_ptr(up.upload(plan.rg_ptr)), rg(up.upload(plan.rg)), rg_ent(up.upload(plan.rg_ent)),
          fast(up.upload(plan.fast)), slow(up.upload(plan.slow)) {}
};

class PanelRun {
  public:
    PanelRun(bem_problem* p, int64_t nt, const DofForecast& f, const double* geo, const double* gbounds,
             const double* crec, SideCopies& up)
        : p_(p), s_(p->stream), nt_(nt), f_(f), geo_(geo), gbounds_(gbounds), crec_(crec), up_(up) {}

    // Groups the row blocks of a numbering with first_dof (N dofs) into panels and allocates the
    // panel buffer, after W (its size is a share of the memory W leaves).
    void layout(const std::vector<int64_t>& first_dof, int64_t N) {
        N_ = N;
        int64_t maxrows = p_->panel_rows;
        if (maxrows <= 0) {
            maxrows = int64_t(p_->tune.panel_fraction * double(available_device_bytes(p_->ctx->device)) / (8.0 * double(nt_)));
            // in steps of 2048 rows, so that a repeat of the same mesh plans the same panels and gets
            // the panel buffer of its predecessor back from the pool
            maxrows = maxrows / 2048 * 2048;
        }
        L_ = layout_panels(first_dof, N, f_, nt_, std::max<int64_t>(maxrows, kTile));
        panels_.clear();
        Ip_.reset();
        // one buffer of the largest panel's size serves all of them (a fresh allocation of tens of
        // GB per panel costs seconds)
        Ip_ = DeviceBuffer(sizeof(double) * size_t(L_.max_elems), s_);
    }

    size_t count() const { return L_.rows.size(); }

    // Queues the far pass of panel pid (panels in order).
    void far(size_t pid) {
        auto P = std::make_unique<Panel>();
        const std::vector<int32_t>& R = L_.rows[pid];
        const int64_t nrows = int64_t(R.size()), t0 = L_.tmin[pid], ncol = nt_ - t0;
        P->ldP = (ncol + 7) / 8 * 8;
        P->rowmap.assign(static_cast<size_t>(nt_), -1);
        for (int64_t r = 0; r < nrows; ++r) P->rowmap[size_t(R[size_t(r)])] = int32_t(r);
        const int64_t nrt = (nrows + kTile - 1) / kTile, nct = (ncol + kTile - 1) / kTile;
        const int64_t ngr = (nrt + kRowGroup - 1) / kRowGroup;
        P->cstart.assign(static_cast<size_t>(std::max<int64_t>(nrt, 1)), 0);
        P->gptr.assign(static_cast<size_t>(ngr) + 1, 0);   // tiles before each group of row tiles
        for (int64_t rb = 0; rb < nrt; ++rb) {
            int64_t cmin = nt_;
            for (int64_t r = rb * kTile; r < std::min<int64_t>(nrows, rb * kTile + kTile); ++r)
                cmin = std::min<int64_t>(cmin, L_.rowfirst[pid][size_t(r)]);
            const int64_t cs = std::min<int64_t>(nct, std::max<int64_t>(0, cmin - t0) / kTile);
            P->cstart[size_t(rb)] = int32_t(cs);
            P->gptr[size_t(rb / kRowGroup) + 1] += nct - cs;
        }
        for (int64_t g = 0; g < ngr; ++g) P->gptr[size_t(g) + 1] += P->gptr[size_t(g)];
        const int64_t nft = P->gptr[size_t(ngr)];
        DeviceBuffer d_rows = up_.upload(R), d_cs = up_.upload(P->cstart), d_gp = up_.upload(P->gptr);
        P->d_rowmap = up_.upload(P->rowmap);
        DeviceBuffer d_ft(sizeof(int2) * size_t(std::max<int64_t>(nft, 1)), s_);
        if (nft > 0) {
            hipLaunchKernelGGL(k_rect_tiles, dim3(unsigned(ngr), unsigned((nct + 255) / 256)), dim3(256), 0, s_,
                               d_cs.as<int32_t>(), d_gp.as<int64_t>(), int32_t(nrt), int32_t(nct), d_ft.as<int2>());
            HIP_CHECK(hipGetLastError());
        }
        P->ef = std::make_unique<EventTimer>(s_);
        if (nft > 0) {
            hipLaunchKernelGGL(k_far_rect, dim3(blocks_for(nft, 4)), dim3(256), 0, s_, geo_, gbounds_, crec_, int32_t(nt_),
                               d_rows.as<int32_t>(), nrows, t0, P->ldP, d_ft.as<int2>(), nft, p_->tune.far_separation,
                               Ip_.as<double>());
            HIP_CHECK(hipGetLastError());
        }
        P->ef->stop();
        if (panels_.size() <= pid) panels_.resize(pid + 1);
        panels_[pid] = std::move(P);
    }

    // Queues the near pairs and the contraction of panel pid, whose far pass is queued.
    template <class Mark>
    void finish(size_t pid, const NearList& near, const PlanDevice& pd, const ContractPlan& plan, const double* dV,
                const double* dgx, const double* dgw, const double* dofJ, float* w32, Mark&& mark) {
        Panel& P = *panels_[pid];
        const int64_t t0 = L_.tmin[pid], ldP = P.ldP;
        // near pairs with a position in this panel (filtered on the host while the far pass runs)
        for (size_t i = 0; i < near.t1.size(); ++i) {
            const int ty = near.type[i];
            const int32_t a = near.t1[i], b = near.t2[i];
            int64_t g1 = -1, g2 = -1;
            if (P.rowmap[size_t(a)] >= 0 && b >= t0) g1 = int64_t(P.rowmap[size_t(a)]) * ldP + (b - t0);
            if (a != b && P.rowmap[size_t(b)] >= 0 && a >= t0) g2 = int64_t(P.rowmap[size_t(b)]) * ldP + (a - t0);
            if (g1 < 0 && g2 < 0) continue;
            P.na[ty].push_back(a);
            P.nb[ty].push_back(b);
            P.nv[ty].insert(P.nv[ty].end(), &near.verts[5 * i], &near.verts[5 * i] + 5);
            P.tgt[ty].push_back(g1);
            P.tgt[ty].push_back(g2);
        }
        DeviceBuffer dv[4], da[4], dbb[4], dt[4];
        for (int ty = 1; ty <= 3; ++ty) {
            if (P.na[ty].empty()) continue;
            dv[ty] = up_.upload(P.nv[ty]);
            da[ty] = up_.upload(P.na[ty]);
            dbb[ty] = up_.upload(P.nb[ty]);
            dt[ty] = up_.upload(P.tgt[ty]);
        }
        P.en = std::make_unique<EventTimer>(s_);
        for (int ty = 1; ty <= 3; ++ty) {
            const int64_t n = int64_t(P.na[ty].size());
            if (n == 0) continue;
            dim3 grid(blocks_for(n, 64)), block(64);
            if (ty == 3)
                hipLaunchKernelGGL(k_near_coincident, grid, block, 0, s_, dV, dv[ty].as<int32_t>(), da[ty].as<int32_t>(), n,
                                   p_->near_order, dgx, dgw, Ip_.as<double>(), ldP, dt[ty].as<int64_t>());
            else if (ty == 2)
                hipLaunchKernelGGL(k_near_edge, grid, block, 0, s_, dV, dv[ty].as<int32_t>(), da[ty].as<int32_t>(),
                                   dbb[ty].as<int32_t>(), n, p_->near_order, dgx, dgw, Ip_.as<double>(), ldP, dt[ty].as<int64_t>());
            else
                hipLaunchKernelGGL(k_near_vertex, grid, block, 0, s_, dV, dv[ty].as<int32_t>(), da[ty].as<int32_t>(),
                                   dbb[ty].as<int32_t>(), n, p_->near_order, dgx, dgw, Ip_.as<double>(), ldP, dt[ty].as<int64_t>());
            HIP_CHECK(hipGetLastError());
        }
        P.en->stop();
        // this panel's tiles of the upper half (the tile lists are sorted by row block)
        const int64_t bd0 = L_.starts[pid], bd1 = L_.starts[pid + 1];
        // The layout puts every row these tiles read in the panel, and their columns at or past the
        // panel's first column; both are checked here, since a miss would read outside the buffer.
        if (cbmin_.empty()) {
            const int64_t ncb = int64_t(plan.cb_ptr.size()) - 1;
            cbmin_.assign(static_cast<size_t>(ncb) + 1, nt_);
            for (int64_t be = ncb - 1; be >= 0; --be)
                cbmin_[size_t(be)] = std::min<int64_t>(cbmin_[size_t(be) + 1], plan.cb_ptr[size_t(be)] < plan.cb_ptr[size_t(be) + 1]
                                                                                ? plan.cb_tri[size_t(plan.cb_ptr[size_t(be)])] : nt_);
        }
        bool fits = cbmin_[size_t(bd0)] >= t0;
        for (int64_t rb = 4 * bd0; fits && rb < 4 * bd1; ++rb)
            for (int32_t g = plan.rg_ptr[size_t(rb)]; g < plan.rg_ptr[size_t(rb) + 1]; ++g)
                fits = fits && P.rowmap[size_t(plan.rg[size_t(g)].x)] >= 0;
        if (!fits) fail(BEM_E_DEVICE, "internal error: a pair-matrix panel lacks entries its contraction reads");
        auto range = [&](const std::vector<int2>& v) {
            auto lo = std::lower_bound(v.begin(), v.end(), int(bd0), [](const int2& x, int b) { return x.x < b; });
            auto hi = std::lower_bound(v.begin(), v.end(), int(bd1), [](const int2& x, int b) { return x.x < b; });
            return std::make_pair(int64_t(lo - v.begin()), int64_t(hi - lo));
        };
        const auto rf = range(plan.fast), rs = range(plan.slow);
        P.ec = std::make_unique<EventTimer>(s_);
        if (rf.second > 0) {
            hipLaunchKernelGGL(k_contract_staged, dim3(unsigned((rf.second + 7) / 8 * 8)), dim3(256), 0, s_, Ip_.as<double>(), ldP,
                               P.d_rowmap.as<int32_t>(), t0, N_, pd.cb_ptr.as<int32_t>(), pd.cb_tri.as<int32_t>(),
                               p_->dof_ptr.as<int64_t>(), pd.col_loc.as<int32_t>(), dofJ, pd.rg_ptr.as<int32_t>(),
                               pd.rg.as<int4>(), pd.rg_ent.as<int2>(), pd.fast.as<int2>() + rf.first, rf.second,
                               p_->W64.as<double>(), w32, p_->ldw);
            HIP_CHECK(hipGetLastError());
        }
        if (rs.second > 0) {
            hipLaunchKernelGGL(k_contract, dim3(unsigned((rs.second + 7) / 8 * 8)), dim3(256), 0, s_, Ip_.as<double>(), ldP,
                               P.d_rowmap.as<int32_t>(), t0, N_, p_->dof_ptr.as<int64_t>(), p_->dof_tri.as<int32_t>(), dofJ,
                               pd.slow.as<int2>() + rs.first, rs.second, p_->W64.as<double>(), w32, p_->ldw);
            HIP_CHECK(hipGetLastError());
        }
        P.ec->stop();
        mark("panel");
    }

    // The event pairs of every panel (far pass, near pairs, contraction, in that order), handed over
    // to be read once the device work has finished.
    std::vector<hipEvent_t> take_events() {
        std::vector<hipEvent_t> ev;
        for (auto& P : panels_) {
            if (!P) continue;
            for (EventTimer* t : {P->ef.get(), P->en.get(), P->ec.get()}) {
                if (!t) continue;
                ev.push_back(t->a);
                ev.push_back(t->b);
                t->a = t->b = nullptr;
            }
        }
        return ev;
    }

  private:
    struct Panel {   // host arrays stay alive until the end: their uploads are asynchronous
        int64_t ldP = 0;
        std::vector<int32_t> rowmap, cstart, nv[4], na[4], nb[4];
        std::vector<int64_t> gptr, tgt[4];
        DeviceBuffer d_rowmap;
        std::unique_ptr<EventTimer> ef, en, ec;
    };
    bem_problem* p_;
    hipStream_t s_;
    int64_t nt_, N_ = 0;
    const DofForecast& f_;
    const double *geo_, *gbounds_, *crec_;
    SideCopies& up_;
    PanelLayout L_;
    std::vector<std::unique_ptr<Panel>> panels_;
    std::vector<int64_t> cbmin_;   // smallest triangle of the column lists from each column block on
    DeviceBuffer Ip_;
};

}  // namespace

void renumber_mesh_device(const double* dV, const int32_t* dT, int64_t nv, int64_t nt, const int32_t* d_vert_user,
                          const int32_t* d_vert_int, const int32_t* d_tri_user, double* Vout, int32_t* Tout, hipStream_t s) {
    const int64_t n = std::max(nv, nt);
    hipLaunchKernelGGL(k_renumber_mesh, dim3(blocks_for(n, 256)), dim3(256), 0, s, dV, dT, nv, nt, d_vert_user, d_vert_int,
                       d_tri_user, Vout, Tout);
    HIP_CHECK(hipGetLastError());
}

void assemble_device(bem_problem* p, const double* Vin, int64_t nv, const int32_t* Tin, int64_t nt,
                     const std::function<void(NearList&)>& analyse, const double* dVin, const int32_t* dTin) {
    const MeshTopo& m = p->topo;
    hipStream_t s = p->stream;
    // BEM_TRACE=1: synchronise and print the wall time of each assembly phase to stderr
    const bool trace = std::getenv("BEM_TRACE") != nullptr;
    auto tlast = std::chrono::steady_clock::now();
    auto mark = [&](const char* what) {
        if (!trace) return;
        HIP_CHECK(hipStreamSynchronize(s));
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "bem-trace assemble %-18s %8.3f ms\n", what, std::chrono::duration<double>(now - tlast).count() * 1e3);
        tlast = now;
    };
    // The geometry and far-field kernels need only coordinates and in-range indices.  They go first,
    // and the host's mesh analysis (sectors, dofs, near list) runs while the device integrates; a
    // mesh the analysis rejects leaves only discarded device work behind.  Indices and referenced
    // coordinates are checked here so that no kernel can read outside the vertex array.
    bool launchable = Vin && Tin && nv > 0 && nt > 0 && nt <= (int64_t(1) << 30);
    if (launchable) {
        std::atomic<bool> bad{false};
        parallel_for(3 * nt, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) {
                const int32_t v = Tin[i];
                if (!(v >= 0 && v < nv && std::isfinite(Vin[3 * v]) && std::isfinite(Vin[3 * v + 1]) &&
                      std::isfinite(Vin[3 * v + 2])))
                    bad = true;
            }
        }, 1 << 16);
        launchable = !bad;
    }
    if (!launchable) {
        NearList unused;
        analyse(unused);   // reports the specific validation error
        fail(BEM_E_INVALID_ARG, "mesh rejected");
    }

    double bary[7][3], w7[7];
    triangle7_rule(bary, w7);
    std::vector<double> hb(&bary[0][0], &bary[0][0] + 21), hw(w7, w7 + 7);

    // the kernels read device copies of the mesh that the call owns (copied from the caller's device
    // arrays, or uploaded), so that the call may return while its kernels still run
    DeviceBuffer dVbuf(sizeof(double) * 3 * nv, s), dTbuf(sizeof(int32_t) * 3 * nt, s);
    HIP_CHECK(hipMemcpyAsync(dVbuf.ptr, dVin ? static_cast<const void*>(dVin) : static_cast<const void*>(Vin), dVbuf.bytes,
                             dVin ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(dTbuf.ptr, dTin ? static_cast<const void*>(dTin) : static_cast<const void*>(Tin), dTbuf.bytes,
                             dTin ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    EventTimer inputs_read(s);   // its end: the caller's device arrays have been read
    inputs_read.stop();
    const double* dVp = dVbuf.as<double>();
    const int32_t* dTp = dTbuf.as<int32_t>();
    DeviceBuffer db = upload(hb, s), dw = upload(hw, s);
    DeviceBuffer geo(sizeof(double) * nt * kGeo, s);
    p->normal = DeviceBuffer(sizeof(double) * nt * 3, s);
    p->area = DeviceBuffer(sizeof(double) * nt, s);
    hipLaunchKernelGGL(k_geometry, dim3(blocks_for(nt, 256)), dim3(256), 0, s, dVp, dTp, nt,
                       db.as<double>(), dw.as<double>(), geo.as<double>(), p->normal.as<double>(), p->area.as<double>());
    HIP_CHECK(hipGetLastError());

    // pair integrals I (nt x ldI), rows padded to 64 bytes so the far kernel's paired stores stay aligned.
    // When the whole matrix does not fit next to W (about 8 N_T^2 + 3 N_T^2 bytes with N ~ N_T / 2),
    // or panels are requested, it is built and contracted panel by panel.
    const int64_t ldI = (nt + 7) / 8 * 8;
    const size_t free_b = available_device_bytes(p->ctx->device);
    const double full_bytes = 8.0 * double(nt) * double(ldI) + 3.0 * double(nt) * double(nt);
    const bool paneled = p->panel_rows > 0 || full_bytes > 0.85 * double(free_b);
    if (paneled && p->has_pairs) fail(BEM_E_INVALID_ARG, "keep_pair_matrix needs the whole pair matrix on the device");
    EventTimer t_far(s);
    // group bounds and column records of the far-field pass (both modes)
    const int64_t ng = (int64_t(nt) + kGrp - 1) / kGrp;
    DeviceBuffer gbounds(sizeof(double) * 4 * std::max<int64_t>(ng, 1), s), crec(sizeof(double) * kRec * std::max<int64_t>(nt, 1), s);
    if (nt > 0) {
        hipLaunchKernelGGL(k_group_bounds, dim3(blocks_for(ng, 256)), dim3(256), 0, s, geo.as<double>(), int32_t(nt),
                           gbounds.as<double>());
        hipLaunchKernelGGL(k_col_records, dim3(blocks_for(nt, 256)), dim3(256), 0, s, geo.as<double>(), gbounds.as<double>(),
                           int32_t(nt), crec.as<double>());
        HIP_CHECK(hipGetLastError());
    }
    if (!paneled) {
        p->ldI = ldI;
        p->I = DeviceBuffer(sizeof(double) * nt * ldI, s);
        const int nb = int((nt + kTile - 1) / kTile);
        // tiles (rb, cb >= rb) in groups of kRowGroup row tiles, column by column within a group (the
        // order of the panels' tile lists, for the same reuse of the column records)
        std::vector<int2> tiles;
        tiles.reserve(size_t(nb) * (nb + 1) / 2);
        for (int g0 = 0; g0 < nb; g0 += kRowGroup)
            for (int cb = g0; cb < nb; ++cb)
                for (int rb = g0; rb < std::min(g0 + kRowGroup, cb + 1); ++rb) tiles.push_back(make_int2(rb, cb));
        DeviceBuffer dtiles = upload(tiles, s);
        HIP_CHECK(hipEventRecord(t_far.a, s));
        const int64_t nti = int64_t(tiles.size());
        hipLaunchKernelGGL(k_far, dim3(blocks_for(nti, 4)), dim3(256), 0, s, geo.as<double>(), gbounds.as<double>(),
                           crec.as<double>(), int32_t(nt), ldI, dtiles.as<int2>(), nti, p->tune.far_separation, p->I.as<double>());
        HIP_CHECK(hipGetLastError());
    }
    t_far.stop();
    // W: every entry, padding columns included, is written by one contraction tile
    auto allocate_w = [&](int64_t n) {
        p->ldw = ((n + 63) / 64) * 64;
        p->W64.reset();
        p->W32.reset();
        p->W64 = DeviceBuffer(sizeof(double) * std::max<int64_t>(n, 1) * p->ldw, s);
        if (p->has_w32) p->W32 = DeviceBuffer(sizeof(float) * std::max<int64_t>(n, 1) * p->ldw, s);
    };
    // panels: the dofs per vertex from counts, then W, the panel layout and the first panel's far
    // pass, all before the sector analysis, which then runs while the device integrates
    SideCopies up(p->ctx, s);
    std::unique_ptr<DofForecast> forecast;
    std::unique_ptr<PanelRun> run;
    if (paneled) {
        forecast = std::make_unique<DofForecast>(forecast_dofs(Tin, nv, nt));
        if (forecast->N > 0) {
            allocate_w(forecast->N);
            matvec_setup(p, s);   // the products' tile lists go with W (only the geometry is queued yet)
            run = std::make_unique<PanelRun>(p, nt, *forecast, geo.as<double>(), gbounds.as<double>(), crec.as<double>(), up);
            run->layout(forecast->first_dof, forecast->N);
            run->far(0);
        }
    }
    mark("geometry+far");

    // host: mesh analysis, near list, and the plans of the near and contraction passes.  If the
    // analysis rejects the mesh, the queued kernels finish before their buffers are released.
    const auto h0 = std::chrono::steady_clock::now();
    NearList near;
    std::vector<int32_t> nv_[4], na_[4], nb_[4];
    ContractPlan plan;
    std::vector<double> gx, gw;
    try {
        analyse(near);
        // the near pairs by kind for the one-shot kernels (panels filter the list themselves), on a
        // thread of its own beside the contraction plan
        std::thread split;
        if (!paneled)
            split = std::thread([&]() {
                for (int ty = 1; ty <= 3; ++ty) {
                    na_[ty].reserve(size_t(near.count[ty]));
                    nb_[ty].reserve(size_t(near.count[ty]));
                    nv_[ty].reserve(size_t(5 * near.count[ty]));
                }
                for (size_t i = 0; i < near.t1.size(); ++i) {
                    const int ty = near.type[i];
                    na_[ty].push_back(near.t1[i]);
                    nb_[ty].push_back(near.t2[i]);
                    nv_[ty].insert(nv_[ty].end(), &near.verts[5 * i], &near.verts[5 * i] + 5);
                }
            });
        try {
            if (m.N > 0) plan = contract_plan(m);
            gauss_legendre01(p->near_order, gx, gw);
        } catch (...) {
            if (split.joinable()) split.join();
            throw;
        }
        if (split.joinable()) split.join();
    } catch (...) {
        (void)hipStreamSynchronize(s);
        throw;
    }
    const int64_t N = m.N;
    p->t_host = std::chrono::duration<double>(std::chrono::steady_clock::now() - h0).count();
    p->n_near = int64_t(near.t1.size());
    mark("host analysis");
    // BEM_PANELS_AFTER_ANALYSIS=1 takes this path for every mesh (for tests of it)
    if (paneled && (N != forecast->N || m.first_dof != forecast->first_dof || std::getenv("BEM_PANELS_AFTER_ANALYSIS"))) {
        // the analysis numbers the dofs otherwise than the forecast: the panels are planned again
        // from its numbering, after the first panel's far pass (now of no use) has finished
        HIP_CHECK(hipStreamSynchronize(s));
        p->panels_replanned = 1;
        run.reset();
        if (N != forecast->N || N == 0) allocate_w(N);
        if (N > 0) {
            if (N != forecast->N) matvec_setup(p, s);
            run = std::make_unique<PanelRun>(p, nt, *forecast, geo.as<double>(), gbounds.as<double>(), crec.as<double>(), up);
            run->layout(m.first_dof, N);
            run->far(0);
        }
    }

    // incidence tables, the contraction plan and the near pairs go up beside the far pass
    p->dof_ptr = up.upload(m.dof_ptr);
    p->dof_tri = up.upload(m.dof_tri);
    p->dof_c = up.upload(m.dof_c);
    DeviceBuffer dof_corner = up.upload(m.dof_corner);
    p->tri_ptr = up.upload(m.tri_ptr);
    p->tri_dof = up.upload(m.tri_dof);
    p->tri_corner = up.upload(m.tri_corner);
    p->tri_c = up.upload(m.tri_c);
    DeviceBuffer dgx = up.upload(gx), dgw = up.upload(gw);
    std::unique_ptr<PlanDevice> pd;
    if (N > 0) pd = std::make_unique<PlanDevice>(plan, up);
    DeviceBuffer dv[4], da[4], dbb[4];
    if (!paneled)
        for (int ty = 1; ty <= 3; ++ty) {
            if (na_[ty].empty()) continue;
            dv[ty] = up.upload(nv_[ty]);
            da[ty] = up.upload(na_[ty]);
            dbb[ty] = up.upload(nb_[ty]);
        }
    // jump vectors
    const int64_t ne = int64_t(m.dof_tri.size());
    DeviceBuffer dofJ(sizeof(double) * 3 * std::max<int64_t>(ne, 1), s);
    if (ne > 0) {
        hipLaunchKernelGGL(k_jump_vectors, dim3(blocks_for(ne, 256)), dim3(256), 0, s, dVp, dTp,
                           p->dof_tri.as<int32_t>(), dof_corner.as<int8_t>(), p->dof_c.as<int8_t>(), p->area.as<double>(), ne,
                           dofJ.as<double>());
        HIP_CHECK(hipGetLastError());
    }

    if (!paneled || N == 0) allocate_w(N);
    float* w32 = p->has_w32 ? p->W32.as<float>() : nullptr;   // the contraction writes both copies
    EventTimer t_near(s), t_contract(s);
    int n_panels = 0;
    if (!paneled) {
        // near pairs, one kernel per kind
        HIP_CHECK(hipEventRecord(t_near.a, s));
        for (int ty = 1; ty <= 3; ++ty) {
            const int64_t n = int64_t(na_[ty].size());
            if (n == 0) continue;
            dim3 grid(blocks_for(n, 64)), block(64);
            if (ty == 3)
                hipLaunchKernelGGL(k_near_coincident, grid, block, 0, s, dVp, dv[ty].as<int32_t>(), da[ty].as<int32_t>(), n,
                                   p->near_order, dgx.as<double>(), dgw.as<double>(), p->I.as<double>(), ldI, nullptr);
            else if (ty == 2)
                hipLaunchKernelGGL(k_near_edge, grid, block, 0, s, dVp, dv[ty].as<int32_t>(), da[ty].as<int32_t>(),
                                   dbb[ty].as<int32_t>(), n, p->near_order, dgx.as<double>(), dgw.as<double>(), p->I.as<double>(), ldI, nullptr);
            else
                hipLaunchKernelGGL(k_near_vertex, grid, block, 0, s, dVp, dv[ty].as<int32_t>(), da[ty].as<int32_t>(),
                                   dbb[ty].as<int32_t>(), n, p->near_order, dgx.as<double>(), dgw.as<double>(), p->I.as<double>(), ldI, nullptr);
            HIP_CHECK(hipGetLastError());
        }
        t_near.stop();
        mark("near");
        HIP_CHECK(hipEventRecord(t_contract.a, s));
        if (N > 0) {
            matvec_setup(p, s);   // its uploads too come before the event the host waits for
            HIP_CHECK(hipEventRecord(t_contract.a, s));
            const int64_t nf = int64_t(plan.fast.size()), ns = int64_t(plan.slow.size());
            if (nf > 0) {
                hipLaunchKernelGGL(k_contract_staged, dim3(unsigned((nf + 7) / 8 * 8)), dim3(256), 0, s, p->I.as<double>(), ldI,
                                   nullptr, int64_t(0), N,
                                   pd->cb_ptr.as<int32_t>(), pd->cb_tri.as<int32_t>(), p->dof_ptr.as<int64_t>(),
                                   pd->col_loc.as<int32_t>(), dofJ.as<double>(), pd->rg_ptr.as<int32_t>(), pd->rg.as<int4>(),
                                   pd->rg_ent.as<int2>(), pd->fast.as<int2>(), nf, p->W64.as<double>(), w32, p->ldw);
                HIP_CHECK(hipGetLastError());
            }
            if (ns > 0) {
                hipLaunchKernelGGL(k_contract, dim3(unsigned((ns + 7) / 8 * 8)), dim3(256), 0, s, p->I.as<double>(), ldI,
                                   nullptr, int64_t(0), N,
                                   p->dof_ptr.as<int64_t>(), p->dof_tri.as<int32_t>(), dofJ.as<double>(), pd->slow.as<int2>(), ns,
                                   p->W64.as<double>(), w32, p->ldw);
                HIP_CHECK(hipGetLastError());
            }
        }
        t_contract.stop();
        mark("contract");
    } else if (run) {
        for (size_t pid = 0; pid < run->count(); ++pid) {
            if (pid > 0) run->far(pid);
            run->finish(pid, near, *pd, plan, dVp, dgx.as<double>(), dgw.as<double>(), dofJ.as<double>(), w32, mark);
        }
        n_panels = int(run->count());
        // The host returns with the panels' device work queued (behind it the host-side work of the
        // next call, e.g. the preconditioner's, overlaps it): every later call on the problem queues
        // behind it on the problem's stream.  The uploads have read their host arrays, the caller's
        // device arrays have been copied, and the phases' device times are read when asked for.
        p->ev_spans = run->take_events();
        HIP_CHECK(hipStreamSynchronize(up.side));
        HIP_CHECK(hipEventSynchronize(inputs_read.b));
    }
    if (run) {
        // panels: nothing more to wait for (above)
    } else if (paneled || N == 0) {   // no dofs
        matvec_setup(p, s);
        HIP_CHECK(hipStreamSynchronize(s));
    } else {
        // The host returns once the inputs are consumed: the event before the contraction follows
        // the last kernel that reads the mesh and the last upload from host memory.  The
        // contraction itself runs on; every later call on the problem queues behind it on the
        // problem's stream, and the calls that read W on other paths synchronise that stream.
        HIP_CHECK(hipEventSynchronize(t_contract.a));
    }
    if (!p->has_pairs) p->I.reset();   // released in stream order, after the contraction
    p->t_far = paneled ? 0.0 : t_far.seconds();    // panels: from p->ev_spans when asked for
    p->t_near = paneled ? 0.0 : t_near.seconds();
    if (paneled || N == 0) {
        p->t_contract = paneled ? 0.0 : t_contract.seconds();
    } else {   // read when the problem's information is first asked for
        p->ev_contract[0] = t_contract.a;
        p->ev_contract[1] = t_contract.b;
        t_contract.a = t_contract.b = nullptr;
    }
    p->n_panels = n_panels;
}

void rhs_device(const bem_problem* p, const double* d_g, int k, double* d_L, hipStream_t s) {
    const int64_t N = p->N;
    if (N == 0) return;
    if (p->topo.dim == 2)
        hipLaunchKernelGGL(k_rhs2d, dim3(blocks_for(N, 256)), dim3(256), 0, s, p->dof_ptr.as<int64_t>(), p->dof_tri.as<int32_t>(),
                           p->dof_c.as<int8_t>(), p->normal.as<double>(), p->area.as<double>(), N, d_g, k, d_L);
    else
        hipLaunchKernelGGL(k_rhs, dim3(blocks_for(N, 256)), dim3(256), 0, s, p->dof_ptr.as<int64_t>(), p->dof_tri.as<int32_t>(),
                           p->dof_c.as<int8_t>(), p->normal.as<double>(), p->area.as<double>(), N, d_g, k, d_L);
    HIP_CHECK(hipGetLastError());
}

void jump_values_device(const bem_problem* p, const double* d_phi, double* d_jump, hipStream_t s) {
    const int64_t nt = p->topo.nt;
    hipLaunchKernelGGL(k_jump_values, dim3(blocks_for(nt, 256)), dim3(256), 0, s, p->tri_ptr.as<int64_t>(), p->tri_dof.as<int32_t>(),
                       p->tri_corner.as<int8_t>(), p->tri_c.as<int8_t>(), nt, p->topo.dim == 2 ? 2 : 3, d_phi, d_jump);
    HIP_CHECK(hipGetLastError());
}

}  // namespace bem
