// The method on segment multiscreens in the plane (paper: Section 2, Experiments 1 and 2; the
// analysis of Sections 3-6 carries over with segments for triangles).  The fundamental solution is
// -log|x - y| / (2 pi) and the surface curl of a jump is its derivative along the segment, so
//
//   W_{d,d'} = sum_{s,s'} D_{s,d} D_{s',d'} K(s,s'),   K(s,s') = -1/(2 pi) int_s int_s' log|x - y|,
//   D_{s,d} = (c_{s,1,d} - c_{s,0,d}) / |s|   (the jump of psi_d is linear on s).
//
// Device work: k_pairs2d forms K for every pair of segments (8-point Gauss-Legendre on both
// segments when they share no end; a segment with itself in closed form; two segments with a
// common end split along the diagonal of their parameter square, the singular factor integrated
// exactly and the remaining regular integrals by 24-point Gauss-Legendre), then k_contract2d forms
// each entry of the upper half of W from the two dofs' star entries and writes it to both halves.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace bem {

namespace {

constexpr double kInv2Pi = 0.15915494309189533576888376337251436;
constexpr int kFarPts = 8;
constexpr int kNearPts = 24;

inline unsigned nblocks(int64_t n, int per) { return unsigned((n + per - 1) / per); }

// int_0^1 log(a h^2 + b h + c) dh for a quadratic that stays positive on [0, 1]
__device__ double log_quadratic(double a, double b, double c, const double* hx, const double* hw) {
    double s = 0.0;
    for (int i = 0; i < kNearPts; ++i) s += hw[i] * log(fma(fma(a, hx[i], b), hx[i], c));
    return s;
}

// K[s][t] and K[t][s] for t >= s: one thread per pair of the upper triangle in 16 x 16 blocks
__global__ __launch_bounds__(256) void k_pairs2d(const double* __restrict__ V, const int32_t* __restrict__ S, int64_t ns,
                                                 const double* __restrict__ gx, const double* __restrict__ gw,
                                                 const double* __restrict__ hx, const double* __restrict__ hw,
                                                 double* __restrict__ K) {
    const int64_t s = int64_t(blockIdx.y) * 16 + threadIdx.y;
    const int64_t t = int64_t(blockIdx.x) * 16 + threadIdx.x;
    if (blockIdx.x < blockIdx.y || s >= ns || t >= ns || t < s) return;
    const int32_t sa = S[2 * s], sb = S[2 * s + 1], ta = S[2 * t], tb = S[2 * t + 1];
    const double xa0 = V[2 * sa], xa1 = V[2 * sa + 1], xb0 = V[2 * sb], xb1 = V[2 * sb + 1];
    const double ya0 = V[2 * ta], ya1 = V[2 * ta + 1], yb0 = V[2 * tb], yb1 = V[2 * tb + 1];
    const double L1 = sqrt((xb0 - xa0) * (xb0 - xa0) + (xb1 - xa1) * (xb1 - xa1));
    const double L2 = sqrt((yb0 - ya0) * (yb0 - ya0) + (yb1 - ya1) * (yb1 - ya1));
    double k;
    if (s == t) {
        k = L1 * L1 * (log(L1) - 1.5);   // int_s int_s log|x - y| in closed form
    } else {
        int pi = -1, pj = -1;   // common end: index in (sa, sb) and in (ta, tb)
        if (sa == ta) { pi = 0; pj = 0; }
        else if (sa == tb) { pi = 0; pj = 1; }
        else if (sb == ta) { pi = 1; pj = 0; }
        else if (sb == tb) { pi = 1; pj = 1; }
        if (pi < 0) {
            double acc = 0.0;
            for (int i = 0; i < kFarPts; ++i) {
                const double x0 = fma(gx[i], xb0 - xa0, xa0), x1 = fma(gx[i], xb1 - xa1, xa1);
                double r = 0.0;
                for (int j = 0; j < kFarPts; ++j) {
                    const double d0 = x0 - fma(gx[j], yb0 - ya0, ya0), d1 = x1 - fma(gx[j], yb1 - ya1, ya1);
                    r = fma(gw[j], log(fma(d0, d0, d1 * d1)), r);
                }
                acc = fma(gw[i], r, acc);
            }
            k = 0.5 * L1 * L2 * acc;   // log|x - y| = log(|x - y|^2) / 2
        } else {
            // directions away from the common end P
            const double e10 = (pi == 0 ? xb0 - xa0 : xa0 - xb0) / L1, e11 = (pi == 0 ? xb1 - xa1 : xa1 - xb1) / L1;
            const double e20 = (pj == 0 ? yb0 - ya0 : ya0 - yb0) / L2, e21 = (pj == 0 ? yb1 - ya1 : ya1 - yb1) / L2;
            const double c = e10 * e20 + e11 * e21;
            // int_0^1 int_0^1 log|L1 a e1 - L2 b e2| with b = a h (a = b h on the other half):
            // each half gives -1/4 + (1/4) int_0^1 log(quadratic in h) dh
            const double A = log_quadratic(L2 * L2, -2.0 * L1 * L2 * c, L1 * L1, hx, hw);
            const double B = log_quadratic(L1 * L1, -2.0 * L1 * L2 * c, L2 * L2, hx, hw);
            k = L1 * L2 * (-0.5 + 0.25 * (A + B));
        }
    }
    k *= -kInv2Pi;   // K = -1/(2 pi) times the integral of log|x - y|
    K[s * ns + t] = k;
    K[t * ns + s] = k;
}

// W[d][e] = W[e][d] = sum over the star entries (s, D) of d and (t, D') of e of D D' K[s][t], e >= d
__global__ __launch_bounds__(256) void k_contract2d(const double* __restrict__ K, int64_t ns, int64_t N,
                                                    const int64_t* __restrict__ dof_ptr, const int32_t* __restrict__ dof_seg,
                                                    const double* __restrict__ dof_D, double* __restrict__ W,
                                                    float* __restrict__ W32, int64_t ldw) {
    const int64_t d = int64_t(blockIdx.y) * 16 + threadIdx.y;
    const int64_t e = int64_t(blockIdx.x) * 16 + threadIdx.x;
    if (blockIdx.x < blockIdx.y || d >= N || e >= ldw || e < d) return;
    double w = 0.0;
    if (e < N) {
        for (int64_t p = dof_ptr[d]; p < dof_ptr[d + 1]; ++p) {
            const double* Kr = K + int64_t(dof_seg[p]) * ns;
            double r = 0.0;
            for (int64_t q = dof_ptr[e]; q < dof_ptr[e + 1]; ++q) r = fma(dof_D[q], Kr[dof_seg[q]], r);
            w = fma(dof_D[p], r, w);
        }
    }
    W[d * ldw + e] = w;   // padding columns e >= N get 0
    if (W32) W32[d * ldw + e] = float(w);
    if (e < N && e != d) {
        W[e * ldw + d] = w;
        if (W32) W32[e * ldw + d] = float(w);
    }
}

}  // namespace

void assemble_2d_device(bem_problem* p, const double* V2, int64_t nv, const int32_t* S, int64_t ns) {
    hipStream_t s = p->stream;
    analyze_segments(V2, nv, S, ns, p->topo);
    const MeshTopo& m = p->topo;
    const int64_t N = m.N;
    p->N = N;
    std::vector<double> gx, gw, hx, hw;
    gauss_legendre01(kFarPts, gx, gw);
    gauss_legendre01(kNearPts, hx, hw);
    std::vector<double> V(V2, V2 + 2 * nv);
    std::vector<int32_t> Sv(S, S + 2 * ns);
    // derivative of each star entry's jump along its segment
    std::vector<double> D(m.dof_tri.size());
    for (size_t q = 0; q < D.size(); ++q)
        D[q] = (m.dof_corner[q] == 1 ? 1.0 : -1.0) * double(m.dof_c[q]) / m.area[m.dof_tri[q]];
    DeviceBuffer dV = upload(V, s), dS = upload(Sv, s), dgx = upload(gx, s), dgw = upload(gw, s), dhx = upload(hx, s),
                 dhw = upload(hw, s), dD = upload(D, s);
    p->normal = upload(m.normal, s);
    p->area = upload(m.area, s);
    p->dof_ptr = upload(m.dof_ptr, s);
    p->dof_tri = upload(m.dof_tri, s);
    p->dof_c = upload(m.dof_c, s);
    p->tri_ptr = upload(m.tri_ptr, s);
    p->tri_dof = upload(m.tri_dof, s);
    p->tri_corner = upload(m.tri_corner, s);
    p->tri_c = upload(m.tri_c, s);
    DeviceBuffer K(sizeof(double) * ns * ns, s);
    {
        const unsigned nb = nblocks(ns, 16);
        hipLaunchKernelGGL(k_pairs2d, dim3(nb, nb), dim3(16, 16), 0, s, dV.as<double>(), dS.as<int32_t>(), ns,
                           dgx.as<double>(), dgw.as<double>(), dhx.as<double>(), dhw.as<double>(), K.as<double>());
        HIP_CHECK(hipGetLastError());
    }
    p->ldw = ((N + 63) / 64) * 64;
    p->W64 = DeviceBuffer(sizeof(double) * std::max<int64_t>(N, 1) * p->ldw, s);
    if (p->has_w32) p->W32 = DeviceBuffer(sizeof(float) * std::max<int64_t>(N, 1) * p->ldw, s);
    if (N > 0) {
        const unsigned nr = nblocks(N, 16), nc = nblocks(p->ldw, 16);
        hipLaunchKernelGGL(k_contract2d, dim3(nc, nr), dim3(16, 16), 0, s, K.as<double>(), ns, N, p->dof_ptr.as<int64_t>(),
                           p->dof_tri.as<int32_t>(), dD.as<double>(), p->W64.as<double>(),
                           p->has_w32 ? p->W32.as<float>() : nullptr, p->ldw);
        HIP_CHECK(hipGetLastError());
    }
    matvec_setup(p, s);
    HIP_CHECK(hipStreamSynchronize(s));   // host vectors above must outlive their uploads
}

}  // namespace bem
