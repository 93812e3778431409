// Dense assembly of the hypersingular Galerkin matrix in surface-curl form (paper: Section 4.3,
// eq. eval_a_phiij with Cor. corW):
//
//   W_{d,d'} = sum_{T,T'} I(T,T') J_{T,d} . J_{T',d'},   I(T,T') = 1/(4 pi) int_T int_T' |x-y|^{-1},
//   J_{T,d} = c_{T,a,d} (x_{a+1} - x_{a+2}) / (2|T|)   (dof d sits at corner a of T).
//
// Pipeline (all on the device):
//   k_geometry      per triangle: unit normal, area, the 7 Gauss points and area-weights
//   k_jump_vectors  per (dof, triangle) incidence: J_{T,d}
//   k_far           7x7 product rule for every pair in 64x64 triangle tiles above the diagonal;
//                   each lane keeps its row triangle's Gauss points in registers while the wave
//                   walks the tile's column triangles, whose points come in through scalar loads
//   k_near_*        Duffy-regularised Gauss-Legendre rules for pairs sharing a triangle, an edge
//                   or a vertex (overwrite the far-rule values of those pairs)
//   k_contract      W = sum over the stars of the two dofs, upper triangle, mirrored
//
// The near rules here are the 4-D Duffy rules of the oracle with the radial variable (and, for
// the coincident and edge cases, the anchor variables) integrated exactly: for the kernel
// 1/|x-y| the integrand is a polynomial of degree <= 2 in those variables, which Gauss-Legendre
// integrates exactly from 2 points on, so dropping them changes nothing but rounding.
#include <cmath>

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

// One wave per 64x64 tile (rb <= cb); 4 waves per block.
__global__ __launch_bounds__(256) void k_far(const double* __restrict__ geo, int32_t nt, int64_t ld,
                                             const int2* __restrict__ tiles, int64_t ntiles,
                                             double* __restrict__ I) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const int2 tc = tiles[tile];
    const int rb = __builtin_amdgcn_readfirstlane(tc.x);
    const int cb = __builtin_amdgcn_readfirstlane(tc.y);
    const int t = rb * kTile + lane;
    const bool valid = t < nt;
    const double* g = geo + int64_t(valid ? t : 0) * kGeo;
    double px[7], py[7], pz[7], pw[7];
#pragma unroll
    for (int p = 0; p < 7; ++p) {
        px[p] = g[3 * p];
        py[p] = g[3 * p + 1];
        pz[p] = g[3 * p + 2];
        pw[p] = g[21 + p];
    }
    const int c0 = cb * kTile;
    const int c1 = min(c0 + kTile, nt);
    for (int tp = c0; tp < c1; ++tp) {
        const double* h = geo + int64_t(tp) * kGeo;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double yx = h[3 * q], yy = h[3 * q + 1], yz = h[3 * q + 2];
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < 7; ++p) {
                const double dx = px[p] - yx, dy = py[p] - yy, dz = pz[p] - yz;
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                s = fma(pw[p], rsqrt_refined(r2), s);
            }
            acc = fma(h[21 + q], s, acc);
        }
        const double val = acc * kInv4Pi;
        if (valid && (rb != cb || t < tp)) {
            I[int64_t(tp) * ld + t] = val;
            I[int64_t(t) * ld + tp] = val;
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
                                  double* __restrict__ I, int64_t ld) {
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
    I[t * ld + t] = acc * (1.0 / 3.0) * 4.0 * ar * ar * kInv4Pi;
}

// Common edge A-B: x - y = w1 (B-A) + w2 (C-B) - w3 (C'-B) with w = (s - s', t, t').  The cone
// {w2, w3 >= 0} is cut into four pieces on which max(w1,0) + max(w3, w2-w1) is linear; on each,
// w = xi b(eta) with b on the unit level set.  The anchor s' and xi integrate to 1/6, leaving
// (1/6) sum_R int int J_R(eta) / |D_R(eta)| d eta, J_R = 1 (square faces) or eta1 (triangular).
__global__ void k_near_edge(const double* __restrict__ V, const int32_t* __restrict__ vs,
                            const int32_t* __restrict__ t1, const int32_t* __restrict__ t2, int64_t n,
                            int ng, const double* __restrict__ gx, const double* __restrict__ gw,
                            double* __restrict__ I, int64_t ld) {
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
    I[a * ld + b] = val;
    I[b * ld + a] = val;
}

// Common vertex A: x^ = xi (1, eta1), y^ = xi (eta2, eta2 eta3) on {s' <= s} and the mirror piece;
// Jacobian xi^3 eta2, the xi integral of xi^2 is 1/3.
__global__ void k_near_vertex(const double* __restrict__ V, const int32_t* __restrict__ vs,
                              const int32_t* __restrict__ t1, const int32_t* __restrict__ t2, int64_t n,
                              int ng, const double* __restrict__ gx, const double* __restrict__ gw,
                              double* __restrict__ I, int64_t ld) {
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
    I[a * ld + b] = val;
    I[b * ld + a] = val;
}

// W[d][e] for d <= e over the stars of d and e, written to both halves (exactly symmetric).
__global__ __launch_bounds__(256) void k_contract(const double* __restrict__ I, int64_t ldI,
                                                  const int64_t* __restrict__ dof_ptr,
                                                  const int32_t* __restrict__ dof_tri,
                                                  const double* __restrict__ dof_J, int64_t N,
                                                  double* __restrict__ W, int64_t ldw) {
    const int64_t bx = blockIdx.x, by = blockIdx.y;
    if (by > bx) return;
    const int64_t d = by * 16 + threadIdx.y;
    const int64_t e = bx * 16 + threadIdx.x;
    if (d >= N || e >= N || d > e) return;
    double sum = 0.0;
    const int64_t e0 = dof_ptr[e], e1 = dof_ptr[e + 1];
    for (int64_t i = dof_ptr[d]; i < dof_ptr[d + 1]; ++i) {
        const double* Irow = I + int64_t(dof_tri[i]) * ldI;
        const double j0 = dof_J[3 * i], j1 = dof_J[3 * i + 1], j2 = dof_J[3 * i + 2];
        for (int64_t k = e0; k < e1; ++k) {
            const double dj = j0 * dof_J[3 * k] + j1 * dof_J[3 * k + 1] + j2 * dof_J[3 * k + 2];
            sum = fma(Irow[dof_tri[k]], dj, sum);
        }
    }
    W[d * ldw + e] = sum;
    W[e * ldw + d] = sum;
}

__global__ void k_f64_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) b[i] = float(a[i]);
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

__global__ void k_jump_values(const int64_t* __restrict__ tri_ptr, const int32_t* __restrict__ tri_dof,
                              const int8_t* __restrict__ tri_corner, const int8_t* __restrict__ tri_c,
                              int64_t nt, const double* __restrict__ phi, double* __restrict__ out) {
    int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    double j[3] = {0.0, 0.0, 0.0};
    for (int64_t e = tri_ptr[t]; e < tri_ptr[t + 1]; ++e) j[tri_corner[e]] += double(tri_c[e]) * phi[tri_dof[e]];
    for (int a = 0; a < 3; ++a) out[3 * t + a] = j[a];
}

inline unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }

struct EventTimer {
    hipEvent_t a, b;
    hipStream_t s;
    explicit EventTimer(hipStream_t st) : s(st) {
        HIP_CHECK(hipEventCreate(&a));
        HIP_CHECK(hipEventCreate(&b));
        HIP_CHECK(hipEventRecord(a, s));
    }
    double stop() {
        HIP_CHECK(hipEventRecord(b, s));
        HIP_CHECK(hipEventSynchronize(b));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, a, b));
        return ms * 1e-3;
    }
    ~EventTimer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

}  // namespace

void assemble_device(bem_problem* p, const NearList& near) {
    const MeshTopo& m = p->topo;
    hipStream_t s = p->stream;
    const int64_t nt = m.nt, N = m.N;

    double bary[7][3], w7[7];
    triangle7_rule(bary, w7);
    std::vector<double> hb(&bary[0][0], &bary[0][0] + 21), hw(w7, w7 + 7);
    std::vector<double> gx, gw;
    gauss_legendre01(p->near_order, gx, gw);

    DeviceBuffer dV = upload(m.V, s), dT = upload(m.T, s);
    DeviceBuffer db = upload(hb, s), dw = upload(hw, s), dgx = upload(gx, s), dgw = upload(gw, s);
    DeviceBuffer geo(sizeof(double) * nt * kGeo);
    p->normal = DeviceBuffer(sizeof(double) * nt * 3);
    p->area = DeviceBuffer(sizeof(double) * nt);
    hipLaunchKernelGGL(k_geometry, dim3(blocks_for(nt, 256)), dim3(256), 0, s, dV.as<double>(), dT.as<int32_t>(), nt,
                       db.as<double>(), dw.as<double>(), geo.as<double>(), p->normal.as<double>(), p->area.as<double>());
    HIP_CHECK(hipGetLastError());

    // incidence tables and jump vectors
    p->dof_ptr = upload(m.dof_ptr, s);
    p->dof_tri = upload(m.dof_tri, s);
    p->dof_c = upload(m.dof_c, s);
    DeviceBuffer dof_corner = upload(m.dof_corner, s);
    p->tri_ptr = upload(m.tri_ptr, s);
    p->tri_dof = upload(m.tri_dof, s);
    p->tri_corner = upload(m.tri_corner, s);
    p->tri_c = upload(m.tri_c, s);
    const int64_t ne = int64_t(m.dof_tri.size());
    DeviceBuffer dofJ(sizeof(double) * 3 * std::max<int64_t>(ne, 1));
    if (ne > 0) {
        hipLaunchKernelGGL(k_jump_vectors, dim3(blocks_for(ne, 256)), dim3(256), 0, s, dV.as<double>(), dT.as<int32_t>(),
                           p->dof_tri.as<int32_t>(), dof_corner.as<int8_t>(), p->dof_c.as<int8_t>(), p->area.as<double>(), ne,
                           dofJ.as<double>());
        HIP_CHECK(hipGetLastError());
    }

    // pair integrals I (nt x nt)
    const int64_t ldI = nt;
    p->I = DeviceBuffer(sizeof(double) * nt * ldI);
    const int nb = int((nt + kTile - 1) / kTile);
    std::vector<int2> tiles;
    tiles.reserve(size_t(nb) * (nb + 1) / 2);
    for (int rb = 0; rb < nb; ++rb)
        for (int cb = rb; cb < nb; ++cb) tiles.push_back(make_int2(rb, cb));
    DeviceBuffer dtiles = upload(tiles, s);
    {
        EventTimer tm(s);
        int64_t nti = int64_t(tiles.size());
        hipLaunchKernelGGL(k_far, dim3(blocks_for(nti, 4)), dim3(256), 0, s, geo.as<double>(), int32_t(nt), ldI,
                           dtiles.as<int2>(), nti, p->I.as<double>());
        HIP_CHECK(hipGetLastError());
        p->t_far = tm.stop();
    }

    // near pairs, one kernel per kind
    {
        std::vector<int32_t> v[4], a[4], b[4];
        for (size_t i = 0; i < near.t1.size(); ++i) {
            int ty = near.type[i];
            a[ty].push_back(near.t1[i]);
            b[ty].push_back(near.t2[i]);
            v[ty].insert(v[ty].end(), &near.verts[5 * i], &near.verts[5 * i] + 5);
        }
        EventTimer tm(s);
        DeviceBuffer dv[4], da[4], dbb[4];
        for (int ty = 1; ty <= 3; ++ty) {
            const int64_t n = int64_t(a[ty].size());
            if (n == 0) continue;
            dv[ty] = upload(v[ty], s);
            da[ty] = upload(a[ty], s);
            dbb[ty] = upload(b[ty], s);
            dim3 grid(blocks_for(n, 64)), block(64);
            if (ty == 3)
                hipLaunchKernelGGL(k_near_coincident, grid, block, 0, s, dV.as<double>(), dv[ty].as<int32_t>(), da[ty].as<int32_t>(), n,
                                   p->near_order, dgx.as<double>(), dgw.as<double>(), p->I.as<double>(), ldI);
            else if (ty == 2)
                hipLaunchKernelGGL(k_near_edge, grid, block, 0, s, dV.as<double>(), dv[ty].as<int32_t>(), da[ty].as<int32_t>(),
                                   dbb[ty].as<int32_t>(), n, p->near_order, dgx.as<double>(), dgw.as<double>(), p->I.as<double>(), ldI);
            else
                hipLaunchKernelGGL(k_near_vertex, grid, block, 0, s, dV.as<double>(), dv[ty].as<int32_t>(), da[ty].as<int32_t>(),
                                   dbb[ty].as<int32_t>(), n, p->near_order, dgx.as<double>(), dgw.as<double>(), p->I.as<double>(), ldI);
            HIP_CHECK(hipGetLastError());
        }
        p->t_near = tm.stop();
    }

    // contraction into W
    p->ldw = ((N + 63) / 64) * 64;
    p->W64 = DeviceBuffer(sizeof(double) * std::max<int64_t>(N, 1) * p->ldw);
    HIP_CHECK(hipMemsetAsync(p->W64.ptr, 0, p->W64.bytes, s));   // padding columns stay zero
    if (N > 0) {
        EventTimer tm(s);
        dim3 grid(blocks_for(N, 16), blocks_for(N, 16)), block(16, 16);
        hipLaunchKernelGGL(k_contract, grid, block, 0, s, p->I.as<double>(), ldI, p->dof_ptr.as<int64_t>(), p->dof_tri.as<int32_t>(),
                           dofJ.as<double>(), N, p->W64.as<double>(), p->ldw);
        HIP_CHECK(hipGetLastError());
        p->t_contract = tm.stop();
    }
    if (p->has_w32) {
        p->W32 = DeviceBuffer(sizeof(float) * std::max<int64_t>(N, 1) * p->ldw);
        hipLaunchKernelGGL(k_f64_to_f32, dim3(4096), dim3(256), 0, s, p->W64.as<double>(), p->W32.as<float>(), N * p->ldw);
        HIP_CHECK(hipGetLastError());
    }
    if (!p->has_pairs) p->I.reset();
    p->mv_xt = DeviceBuffer(sizeof(double) * 16 * p->ldw);
    p->mv_partial = DeviceBuffer(sizeof(double) * 16 * 16 * p->ldw);
    HIP_CHECK(hipStreamSynchronize(s));
}

void rhs_device(const bem_problem* p, const double* d_g, int k, double* d_L, hipStream_t s) {
    const int64_t N = p->N;
    if (N == 0) return;
    hipLaunchKernelGGL(k_rhs, dim3(blocks_for(N, 256)), dim3(256), 0, s, p->dof_ptr.as<int64_t>(), p->dof_tri.as<int32_t>(),
                       p->dof_c.as<int8_t>(), p->normal.as<double>(), p->area.as<double>(), N, d_g, k, d_L);
    HIP_CHECK(hipGetLastError());
}

void jump_values_device(const bem_problem* p, const double* d_phi, double* d_jump, hipStream_t s) {
    const int64_t nt = p->topo.nt;
    hipLaunchKernelGGL(k_jump_values, dim3(blocks_for(nt, 256)), dim3(256), 0, s, p->tri_ptr.as<int64_t>(), p->tri_dof.as<int32_t>(),
                       p->tri_corner.as<int8_t>(), p->tri_c.as<int8_t>(), nt, d_phi, d_jump);
    HIP_CHECK(hipGetLastError());
}

}  // namespace bem
