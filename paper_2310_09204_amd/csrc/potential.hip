// Double-layer potential of the discrete solution at points off the screen (paper: Lemma repDL,
// eq. formulaDL).  The two sides of a triangle T carry the normals -n_T and +n_T, so their traces
// combine into the jump [u]_T = gamma_+ u - gamma_- u (linear on T, corner values from the jump
// coefficients) and
//
//   U(x) = sum_T int_T n_T . (x - y) / (4 pi |x - y|^3) [u]_T(y) dsigma(y),
//
// taken with the 7-point rule of the far field on every triangle (accurate for targets a few mesh
// sizes away from the screen; no refinement for closer ones).
//
// Device work: the per-triangle records (unit normal, Gauss points, n . y) are built once per
// problem; per call, the jump values of each column, the point densities, then one thread per
// target walks a chunk of triangles (their data through scalar loads) for up to 16 columns at once,
// and a last kernel sums the chunks in a fixed order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace bem {

namespace {

constexpr int kRecDL = 32;   // n (3), pad, then 7 x (y0, y1, y2, n . y)
constexpr int kCols = 16;    // columns per pass
constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

inline unsigned nblocks(int64_t n, int per) { return unsigned((n + per - 1) / per); }

// dens[(t * 7 + p) * kCols + c] = area w_p / (4 pi) * [u_c]_T(y_p) / 8 for the kc columns of this
// pass (the 1/8 belongs to the reciprocal-cube step of the target kernel)
__global__ void k_dl_density(const double* __restrict__ jump, int64_t nt, int kc, const double* __restrict__ area,
                             const double* __restrict__ rule, double* __restrict__ dens) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= nt * 7) return;
    const int64_t t = e / 7;
    const int p = int(e % 7);
    const double s = area[t] * rule[21 + p] * kInv4Pi * 0.125;
    for (int c = 0; c < kCols; ++c) {
        double v = 0.0;
        if (c < kc) {
            const double* j = jump + (int64_t(c) * nt + t) * 3;
            v = s * (rule[3 * p] * j[0] + rule[3 * p + 1] * j[1] + rule[3 * p + 2] * j[2]);
        }
        dens[e * kCols + c] = v;
    }
}

// part[(chunk * kCols + c) * m + i] = the chunk's share of U_c(x_i)
template <int KC>
__global__ __launch_bounds__(256) void k_double_layer(const double* __restrict__ rec, const double* __restrict__ dens,
                                                      int64_t nt, int64_t tchunk, const double* __restrict__ X, int64_t m,
                                                      double* __restrict__ part) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    const int64_t t0 = chunk * tchunk, t1 = min<int64_t>(nt, t0 + tchunk);
    const int64_t ii = i < m ? i : 0;
    const double x0 = X[3 * ii], x1 = X[3 * ii + 1], x2 = X[3 * ii + 2];
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const double* r = rec + t * kRecDL;
        const double nx = fma(r[0], x0, fma(r[1], x1, r[2] * x2));
        const double* d = dens + t * 7 * kCols;
#pragma unroll
        for (int p = 0; p < 7; ++p) {
            const double* y = r + 4 + 4 * p;
            const double d0 = x0 - y[0], d1 = x1 - y[1], d2 = x2 - y[2];
            const double r2 = fma(d0, d0, fma(d1, d1, d2 * d2));
            // 2/|x - y| = h (3 - r2 h^2) after one Newton step from the hardware estimate h; its cube
            // is 8/|x - y|^3, the 8 taken out of the densities
            const double h = __builtin_amdgcn_rsq(r2);
            const double q = h * fma(-r2, h * h, 3.0);
            const double g = (nx - y[3]) * (q * q * q);
#pragma unroll
            for (int c = 0; c < KC; ++c) acc[c] = fma(g, d[p * kCols + c], acc[c]);
        }
    }
    if (i < m) {
#pragma unroll
        for (int c = 0; c < KC; ++c) part[(chunk * kCols + c) * m + i] = acc[c];
    }
}

__global__ void k_dl_reduce(const double* __restrict__ part, int64_t nchunk, int kc, int64_t m, double* __restrict__ out) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= m || c >= kc) return;
    double s = 0.0;
    for (int64_t ch = 0; ch < nchunk; ++ch) s += part[(ch * kCols + c) * m + i];
    out[int64_t(c) * m + i] = s;
}

// Segment meshes: U(x) = sum_s int_s n_s . (x - y) / (2 pi |x - y|^2) [u]_s(y) dy with 8-point
// Gauss-Legendre on every segment.  rec2[s]: n (2), then 8 x (y0, y1, n . y); dens2[(s * 8 + p) *
// kCols + c] = w_p |s| / (2 pi) [u_c]_s(y_p).
constexpr int kRec2 = 26;
constexpr int kPts2 = 8;

__global__ void k_dl_density2d(const double* __restrict__ jump, int64_t ns, int kc, const double* __restrict__ length,
                               const double* __restrict__ gx, const double* __restrict__ gw, double* __restrict__ dens) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= ns * kPts2) return;
    const int64_t t = e / kPts2;
    const int p = int(e % kPts2);
    const double s = gw[p] * length[t] * 0.15915494309189533576888376337251436;
    for (int c = 0; c < kCols; ++c) {
        double v = 0.0;
        if (c < kc) {
            const double* j = jump + (int64_t(c) * ns + t) * 2;
            v = s * fma(gx[p], j[1] - j[0], j[0]);
        }
        dens[e * kCols + c] = v;
    }
}

template <int KC>
__global__ __launch_bounds__(256) void k_double_layer2d(const double* __restrict__ rec, const double* __restrict__ dens,
                                                        int64_t ns, int64_t tchunk, const double* __restrict__ X, int64_t m,
                                                        double* __restrict__ part) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    const int64_t t0 = chunk * tchunk, t1 = min<int64_t>(ns, t0 + tchunk);
    const int64_t ii = i < m ? i : 0;
    const double x0 = X[3 * ii], x1 = X[3 * ii + 1];
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const double* r = rec + t * kRec2;
        const double nx = fma(r[0], x0, r[1] * x1);
        const double* d = dens + t * kPts2 * kCols;
#pragma unroll
        for (int p = 0; p < kPts2; ++p) {
            const double* y = r + 2 + 3 * p;
            const double d0 = x0 - y[0], d1 = x1 - y[1];
            const double g = (nx - y[2]) / fma(d0, d0, d1 * d1);
#pragma unroll
            for (int c = 0; c < KC; ++c) acc[c] = fma(g, d[p * kCols + c], acc[c]);
        }
    }
    if (i < m) {
#pragma unroll
        for (int c = 0; c < KC; ++c) part[(chunk * kCols + c) * m + i] = acc[c];
    }
}

}  // namespace

namespace {

void double_layer_2d(bem_problem* p, const double* d_phi, int k, const double* d_X, int64_t m, double* d_U, hipStream_t s) {
    const MeshTopo& f = p->topo;
    const int64_t ns = f.nt, N = p->N;
    std::vector<double> gx, gw;
    gauss_legendre01(kPts2, gx, gw);
    if (!p->dl_rec.ptr) {
        std::vector<double> rec(size_t(ns) * kRec2, 0.0);
        for (int64_t t = 0; t < ns; ++t) {
            double* r = &rec[size_t(t) * kRec2];
            const double n0 = f.normal[3 * t], n1 = f.normal[3 * t + 1];
            r[0] = n0;
            r[1] = n1;
            const double* a = &f.V[3 * int64_t(f.S[2 * t])];
            const double* b = &f.V[3 * int64_t(f.S[2 * t + 1])];
            for (int q = 0; q < kPts2; ++q) {
                const double y0 = a[0] + gx[q] * (b[0] - a[0]), y1 = a[1] + gx[q] * (b[1] - a[1]);
                r[2 + 3 * q] = y0;
                r[3 + 3 * q] = y1;
                r[4 + 3 * q] = n0 * y0 + n1 * y1;
            }
        }
        std::vector<double> rule(gx);
        rule.insert(rule.end(), gw.begin(), gw.end());
        p->dl_rec = upload(rec, s);
        p->dl_rule = upload(rule, s);
        HIP_CHECK(hipStreamSynchronize(s));
    }
    const int64_t tblocks = (m + 255) / 256;
    int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>((ns + 63) / 64, (2048 + tblocks - 1) / tblocks));
    const int64_t tchunk = (ns + nchunk - 1) / nchunk;
    nchunk = (ns + tchunk - 1) / tchunk;
    DeviceBuffer jump(sizeof(double) * 2 * ns * kCols, s), dens(sizeof(double) * ns * kPts2 * kCols, s);
    DeviceBuffer part(sizeof(double) * nchunk * kCols * m, s);
    const double* rule = p->dl_rule.as<double>();
    for (int c0 = 0; c0 < k; c0 += kCols) {
        const int kc = std::min(kCols, k - c0);
        for (int c = 0; c < kc; ++c)
            jump_values_device(p, d_phi + int64_t(c0 + c) * N, jump.as<double>() + int64_t(c) * ns * 2, s);
        hipLaunchKernelGGL(k_dl_density2d, dim3(nblocks(ns * kPts2, 256)), dim3(256), 0, s, jump.as<double>(), ns, kc,
                           p->area.as<double>(), rule, rule + kPts2, dens.as<double>());
        const dim3 grid{static_cast<unsigned>(tblocks), static_cast<unsigned>(nchunk)};
        const double* rec = p->dl_rec.as<double>();
        if (kc == 1)
            hipLaunchKernelGGL(k_double_layer2d<1>, grid, dim3(256), 0, s, rec, dens.as<double>(), ns, tchunk, d_X, m, part.as<double>());
        else if (kc <= 4)
            hipLaunchKernelGGL(k_double_layer2d<4>, grid, dim3(256), 0, s, rec, dens.as<double>(), ns, tchunk, d_X, m, part.as<double>());
        else
            hipLaunchKernelGGL(k_double_layer2d<16>, grid, dim3(256), 0, s, rec, dens.as<double>(), ns, tchunk, d_X, m, part.as<double>());
        hipLaunchKernelGGL(k_dl_reduce, dim3(nblocks(m, 256), unsigned(kc)), dim3(256), 0, s, part.as<double>(), nchunk, kc, m,
                           d_U + int64_t(c0) * m);
        HIP_CHECK(hipGetLastError());
    }
}

}  // namespace

void double_layer_device(bem_problem* p, const double* d_phi, int k, const double* d_X, int64_t m, double* d_U,
                         hipStream_t s) {
    const MeshTopo& f = p->topo;
    const int64_t nt = f.nt, N = p->N;
    if (m == 0 || k == 0) return;
    if (f.dim == 2) {
        double_layer_2d(p, d_phi, k, d_X, m, d_U, s);
        return;
    }
    if (!p->dl_rec.ptr) {
        // records of the 7-point rule on every triangle (host, once per problem)
        double bary[7][3], w7[7];
        triangle7_rule(bary, w7);
        std::vector<double> rec(size_t(std::max<int64_t>(nt, 1)) * kRecDL, 0.0);
        for (int64_t t = 0; t < nt; ++t) {
            double* r = &rec[size_t(t) * kRecDL];
            const double* n = &f.normal[3 * t];
            for (int a = 0; a < 3; ++a) r[a] = n[a];
            for (int q = 0; q < 7; ++q) {
                double y[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < 3; ++a)
                    for (int e = 0; e < 3; ++e) y[e] += bary[q][a] * f.V[3 * int64_t(f.T[3 * t + a]) + e];
                for (int e = 0; e < 3; ++e) r[4 + 4 * q + e] = y[e];
                r[4 + 4 * q + 3] = n[0] * y[0] + n[1] * y[1] + n[2] * y[2];
            }
        }
        std::vector<double> rule(28);
        for (int q = 0; q < 7; ++q) {
            for (int a = 0; a < 3; ++a) rule[3 * q + a] = bary[q][a];
            rule[21 + q] = w7[q];
        }
        p->dl_rec = upload(rec, s);
        p->dl_rule = upload(rule, s);
        HIP_CHECK(hipStreamSynchronize(s));   // the host vectors go out of scope
    }
    if (nt == 0) {
        std::vector<double> z(size_t(k) * m, 0.0);
        HIP_CHECK(hipMemcpyAsync(d_U, z.data(), sizeof(double) * z.size(), hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
        return;
    }
    // triangle chunks: enough blocks to fill the chip (about 2048), at least 64 triangles each
    const int64_t tblocks = (m + 255) / 256;
    int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>((nt + 63) / 64, (2048 + tblocks - 1) / tblocks));
    const int64_t tchunk = (nt + nchunk - 1) / nchunk;
    nchunk = (nt + tchunk - 1) / tchunk;
    DeviceBuffer jump(sizeof(double) * 3 * nt * kCols, s), dens(sizeof(double) * nt * 7 * kCols, s);
    DeviceBuffer part(sizeof(double) * nchunk * kCols * m, s);
    for (int c0 = 0; c0 < k; c0 += kCols) {
        const int kc = std::min(kCols, k - c0);
        for (int c = 0; c < kc; ++c)
            jump_values_device(p, d_phi + int64_t(c0 + c) * N, jump.as<double>() + int64_t(c) * nt * 3, s);
        hipLaunchKernelGGL(k_dl_density, dim3(nblocks(nt * 7, 256)), dim3(256), 0, s, jump.as<double>(), nt, kc,
                           p->area.as<double>(), p->dl_rule.as<double>(), dens.as<double>());
        const dim3 grid{static_cast<unsigned>(tblocks), static_cast<unsigned>(nchunk)};
        const double* rec = p->dl_rec.as<double>();
        if (kc == 1)
            hipLaunchKernelGGL(k_double_layer<1>, grid, dim3(256), 0, s, rec, dens.as<double>(), nt, tchunk, d_X, m, part.as<double>());
        else if (kc <= 2)
            hipLaunchKernelGGL(k_double_layer<2>, grid, dim3(256), 0, s, rec, dens.as<double>(), nt, tchunk, d_X, m, part.as<double>());
        else if (kc <= 4)
            hipLaunchKernelGGL(k_double_layer<4>, grid, dim3(256), 0, s, rec, dens.as<double>(), nt, tchunk, d_X, m, part.as<double>());
        else if (kc <= 8)
            hipLaunchKernelGGL(k_double_layer<8>, grid, dim3(256), 0, s, rec, dens.as<double>(), nt, tchunk, d_X, m, part.as<double>());
        else
            hipLaunchKernelGGL(k_double_layer<16>, grid, dim3(256), 0, s, rec, dens.as<double>(), nt, tchunk, d_X, m, part.as<double>());
        hipLaunchKernelGGL(k_dl_reduce, dim3(nblocks(m, 256), unsigned(kc)), dim3(256), 0, s, part.as<double>(), nchunk, kc, m,
                           d_U + int64_t(c0) * m);
        HIP_CHECK(hipGetLastError());
    }
}

}  // namespace bem
