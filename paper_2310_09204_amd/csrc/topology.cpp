// Host-side analysis of a polygonal multiscreen mesh: validation, generalized vertices
// (sectors), jump-basis degrees of freedom, jump coefficients and the near-pair list.
//
// Paper, Section 4.2: around vertex x_i the complement of Gamma splits into q_i connected sectors
// (components of the star graph G(x_i), eqs. defCurlyHOmega/defCurlyHGamma).  The jump basis is
// psi_{i,j} = phi_{i,j} - phi_{i,q_i}, j < q_i (eqs. defCurlyHtildeGamma, defYij).  Section 4.3
// evaluates everything on oriented triangles (T, side); which sides share a sector at a vertex
// is what the sets alpha_{k,l} (eq. defAlphaij) record.
//
// Surface-only construction used here: every (triangle, corner, side) is a node of one global
// union-find.  Around each edge the incident triangles are ordered by angle; the side of a
// triangle facing the next triangle is merged with that triangle's side facing back (at both
// endpoints of the edge); at a free edge the two sides of its triangle are merged.  The classes
// at a vertex are its sectors.  Because the union keeps the smaller node as root, each root is
// the smallest member, i.e. the (triangle index, + before -) first side of the sector, which is
// the canonical label order.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace bem {

namespace {

struct DisjointSets {
    std::vector<int64_t> parent;
    explicit DisjointSets(int64_t n) : parent(n) { std::iota(parent.begin(), parent.end(), int64_t(0)); }
    int64_t root(int64_t x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    }
    void join(int64_t a, int64_t b) {
        a = root(a);
        b = root(b);
        if (a == b) return;
        if (a < b) parent[b] = a; else parent[a] = b;
    }
};

using Vec3 = std::array<double, 3>;

inline Vec3 at(const std::vector<double>& V, int64_t i) { return {V[3 * i], V[3 * i + 1], V[3 * i + 2]}; }
inline Vec3 minus(const Vec3& a, const Vec3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline double dot3(const Vec3& a, const Vec3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline Vec3 cross3(const Vec3& a, const Vec3& b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
inline double norm3(const Vec3& a) { return std::sqrt(dot3(a, a)); }

// node ids of the two union-finds
inline int64_t side_node(int64_t t, int a, int s) { return (t * 3 + a) * 2 + s; }
inline int64_t corner_node(int64_t t, int a) { return t * 3 + a; }

}  // namespace

void analyze_mesh(const double* Vin, int64_t nv, const int32_t* Tin, int64_t nt, MeshTopo& m) {
    if (!Vin || !Tin || nv <= 0 || nt <= 0) fail(BEM_E_INVALID_ARG, "empty mesh");
    if (nt > (int64_t(1) << 30)) fail(BEM_E_INVALID_ARG, "too many triangles");
    m = MeshTopo();
    m.nv = nv;
    m.nt = nt;
    m.V.assign(Vin, Vin + 3 * nv);
    m.T.assign(Tin, Tin + 3 * nt);
    const auto& V = m.V;
    const auto& T = m.T;

    for (int64_t t = 0; t < nt; ++t) {
        for (int a = 0; a < 3; ++a) {
            int32_t v = T[3 * t + a];
            if (v < 0 || v >= nv) fail(BEM_E_INVALID_ARG, "triangle " + std::to_string(t) + " has a vertex index out of range");
            if (!std::isfinite(V[3 * v]) || !std::isfinite(V[3 * v + 1]) || !std::isfinite(V[3 * v + 2]))
                fail(BEM_E_INVALID_ARG, "non-finite vertex coordinate");
        }
        if (T[3 * t] == T[3 * t + 1] || T[3 * t + 1] == T[3 * t + 2] || T[3 * t] == T[3 * t + 2])
            fail(BEM_E_DEGENERATE, "triangle " + std::to_string(t) + " repeats a vertex");
    }

    // ---- element geometry --------------------------------------------------------------------
    m.normal.resize(3 * nt);
    m.area.resize(nt);
    for (int64_t t = 0; t < nt; ++t) {
        Vec3 x0 = at(V, T[3 * t]), x1 = at(V, T[3 * t + 1]), x2 = at(V, T[3 * t + 2]);
        Vec3 e1 = minus(x1, x0), e2 = minus(x2, x0), e3 = minus(x2, x1);
        Vec3 c = cross3(e1, e2);
        double tw = norm3(c);
        double scale = std::max({dot3(e1, e1), dot3(e2, e2), dot3(e3, e3)});
        if (!(tw > 1e-12 * scale)) fail(BEM_E_DEGENERATE, "triangle " + std::to_string(t) + " has zero area");
        for (int k = 0; k < 3; ++k) m.normal[3 * t + k] = c[k] / tw;
        m.area[t] = 0.5 * tw;
    }

    // ---- repeated vertices (by coordinates) and repeated triangles ------------------------------
    {
        std::vector<char> used(nv, 0);
        for (int64_t i = 0; i < 3 * nt; ++i) used[T[i]] = 1;
        std::vector<int64_t> order;
        for (int64_t v = 0; v < nv; ++v) if (used[v]) order.push_back(v);
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
            for (int k = 0; k < 3; ++k)
                if (V[3 * a + k] != V[3 * b + k]) return V[3 * a + k] < V[3 * b + k];
            return a < b;
        });
        for (size_t i = 1; i < order.size(); ++i) {
            int64_t a = order[i - 1], b = order[i];
            if (V[3 * a] == V[3 * b] && V[3 * a + 1] == V[3 * b + 1] && V[3 * a + 2] == V[3 * b + 2])
                fail(BEM_E_MESH_NONCONFORMING, "vertices " + std::to_string(a) + " and " + std::to_string(b) + " coincide");
        }
        std::vector<std::array<int32_t, 3>> tri(nt);
        for (int64_t t = 0; t < nt; ++t) {
            tri[t] = {T[3 * t], T[3 * t + 1], T[3 * t + 2]};
            std::sort(tri[t].begin(), tri[t].end());
        }
        std::sort(tri.begin(), tri.end());
        for (int64_t t = 1; t < nt; ++t)
            if (tri[t] == tri[t - 1]) fail(BEM_E_MESH_NONCONFORMING, "repeated triangle");
    }

    // ---- edges --------------------------------------------------------------------------------
    struct EdgeRec { int32_t lo, hi; int32_t t; };
    std::vector<EdgeRec> edges;
    edges.reserve(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int a = 0; a < 3; ++a) {
            int32_t i = T[3 * t + a], j = T[3 * t + (a + 1) % 3];
            edges.push_back({std::min(i, j), std::max(i, j), int32_t(t)});
        }
    std::sort(edges.begin(), edges.end(), [](const EdgeRec& x, const EdgeRec& y) {
        if (x.lo != y.lo) return x.lo < y.lo;
        if (x.hi != y.hi) return x.hi < y.hi;
        return x.t < y.t;
    });

    auto corner_of = [&](int64_t t, int32_t v) -> int {
        for (int a = 0; a < 3; ++a) if (T[3 * t + a] == v) return a;
        return -1;
    };

    DisjointSets sides(6 * nt), corners(3 * nt);
    struct Item { double theta; int32_t t; Vec3 d; };
    std::vector<Item> fan;
    for (size_t b = 0; b < edges.size();) {
        size_t e = b;
        while (e < edges.size() && edges[e].lo == edges[b].lo && edges[e].hi == edges[b].hi) ++e;
        const int32_t lo = edges[b].lo, hi = edges[b].hi;
        const int32_t ends[2] = {lo, hi};
        for (size_t k = b + 1; k < e; ++k)
            for (int32_t v : ends) corners.join(corner_node(edges[b].t, corner_of(edges[b].t, v)),
                                                corner_node(edges[k].t, corner_of(edges[k].t, v)));
        if (e - b == 1) {
            int32_t t = edges[b].t;
            for (int32_t v : ends) {
                int a = corner_of(t, v);
                sides.join(side_node(t, a, 0), side_node(t, a, 1));
            }
        } else {
            Vec3 axis = minus(at(V, hi), at(V, lo));
            double al = norm3(axis);
            for (auto& c : axis) c /= al;
            fan.clear();
            for (size_t k = b; k < e; ++k) {
                int32_t t = edges[k].t;
                int32_t third = T[3 * t] + T[3 * t + 1] + T[3 * t + 2] - lo - hi;
                Vec3 d = minus(at(V, third), at(V, lo));
                double along = dot3(d, axis);
                for (int c = 0; c < 3; ++c) d[c] -= along * axis[c];
                double dn = norm3(d);
                for (auto& c : d) c /= dn;
                fan.push_back({0.0, t, d});
            }
            const Vec3 b1 = fan[0].d;
            const Vec3 b2 = cross3(axis, b1);
            for (auto& it : fan) {
                double th = std::atan2(dot3(it.d, b2), dot3(it.d, b1));
                it.theta = th < 0 ? th + 2.0 * M_PI : th;
            }
            std::sort(fan.begin(), fan.end(), [](const Item& x, const Item& y) { return x.theta < y.theta; });
            const size_t nf = fan.size();
            for (size_t k = 0; k < nf; ++k) {
                double gap = (k + 1 < nf) ? fan[k + 1].theta - fan[k].theta : fan[0].theta + 2.0 * M_PI - fan[k].theta;
                if (gap < 1e-9) fail(BEM_E_MESH_NONCONFORMING, "two triangles at edge (" + std::to_string(lo) + "," + std::to_string(hi) + ") lie in the same half-plane");
            }
            for (size_t k = 0; k < nf; ++k) {
                const Item& A = fan[k];
                const Item& B = fan[(k + 1) % nf];
                // side facing increasing angle: '+' (0) iff n_T . (axis x d_T) > 0
                Vec3 na = {m.normal[3 * A.t], m.normal[3 * A.t + 1], m.normal[3 * A.t + 2]};
                Vec3 nb = {m.normal[3 * B.t], m.normal[3 * B.t + 1], m.normal[3 * B.t + 2]};
                int inc_a = dot3(na, cross3(axis, A.d)) > 0 ? 0 : 1;
                int inc_b = dot3(nb, cross3(axis, B.d)) > 0 ? 0 : 1;
                int dec_b = 1 - inc_b;
                for (int32_t v : ends)
                    sides.join(side_node(A.t, corner_of(A.t, v), inc_a), side_node(B.t, corner_of(B.t, v), dec_b));
            }
        }
        b = e;
    }

    // ---- per-vertex corners (counting sort) -----------------------------------------------------
    std::vector<int64_t> vptr(nv + 1, 0);
    for (int64_t i = 0; i < 3 * nt; ++i) ++vptr[T[i] + 1];
    for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int64_t> vcorner(3 * nt);
    {
        std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int a = 0; a < 3; ++a) vcorner[fill[T[3 * t + a]]++] = corner_node(t, a);
    }

    m.q.assign(nv, 0);
    m.sector.assign(6 * nt, -1);
    std::vector<int64_t> roots;
    for (int64_t v = 0; v < nv; ++v) {
        if (vptr[v] == vptr[v + 1]) continue;
        int64_t r0 = corners.root(vcorner[vptr[v]]);
        for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k)
            if (corners.root(vcorner[k]) != r0)
                fail(BEM_E_POINT_CONTACT, "point contact at vertex " + std::to_string(v));
        roots.clear();
        for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k)
            for (int s = 0; s < 2; ++s) roots.push_back(sides.root(vcorner[k] * 2 + s));
        std::sort(roots.begin(), roots.end());
        roots.erase(std::unique(roots.begin(), roots.end()), roots.end());
        m.q[v] = int32_t(roots.size());
        for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
            int64_t c = vcorner[k];
            for (int s = 0; s < 2; ++s) {
                int64_t r = sides.root(c * 2 + s);
                m.sector[c * 2 + s] = int32_t(std::lower_bound(roots.begin(), roots.end(), r) - roots.begin());
            }
        }
    }

    // ---- dofs -----------------------------------------------------------------------------------
    m.first_dof.assign(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) m.first_dof[v + 1] = m.first_dof[v] + std::max(0, m.q[v] - 1);
    m.N = m.first_dof[nv];
    m.dof_vertex.resize(m.N);
    m.dof_sector.resize(m.N);
    for (int64_t v = 0; v < nv; ++v)
        for (int64_t d = m.first_dof[v]; d < m.first_dof[v + 1]; ++d) {
            m.dof_vertex[d] = int32_t(v);
            m.dof_sector[d] = int32_t(d - m.first_dof[v]);
        }

    // ---- jump coefficients: trace of psi_{v,j} on side s at the corner is +1 if the side is in
    //      sector j, -1 if it is in the reference sector q_v - 1, else 0; c = s_+ - s_-  ---------
    m.tri_ptr.assign(nt + 1, 0);
    m.tri_dof.clear(); m.tri_corner.clear(); m.tri_c.clear();
    for (int64_t t = 0; t < nt; ++t) {
        for (int a = 0; a < 3; ++a) {
            int32_t v = T[3 * t + a];
            int32_t qv = m.q[v];
            int32_t sp = m.sector[side_node(t, a, 0)], sm = m.sector[side_node(t, a, 1)];
            for (int32_t j = 0; j + 1 < qv; ++j) {
                int c = ((sp == j) ? 1 : (sp == qv - 1 ? -1 : 0)) - ((sm == j) ? 1 : (sm == qv - 1 ? -1 : 0));
                if (c == 0) continue;
                m.tri_dof.push_back(int32_t(m.first_dof[v] + j));
                m.tri_corner.push_back(int8_t(a));
                m.tri_c.push_back(int8_t(c));
            }
        }
        m.tri_ptr[t + 1] = int64_t(m.tri_dof.size());
    }
    const int64_t ne = int64_t(m.tri_dof.size());
    m.dof_ptr.assign(m.N + 1, 0);
    for (int64_t e = 0; e < ne; ++e) ++m.dof_ptr[m.tri_dof[e] + 1];
    for (int64_t d = 0; d < m.N; ++d) m.dof_ptr[d + 1] += m.dof_ptr[d];
    m.dof_tri.resize(ne); m.dof_corner.resize(ne); m.dof_c.resize(ne);
    {
        std::vector<int64_t> fill(m.dof_ptr.begin(), m.dof_ptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int64_t e = m.tri_ptr[t]; e < m.tri_ptr[t + 1]; ++e) {
                int64_t pos = fill[m.tri_dof[e]]++;
                m.dof_tri[pos] = int32_t(t);
                m.dof_corner[pos] = m.tri_corner[e];
                m.dof_c[pos] = m.tri_c[e];
            }
    }
}

void build_near_list(const MeshTopo& m, NearList& out) {
    out = NearList();
    const int64_t nt = m.nt, nv = m.nv;
    const auto& T = m.T;
    std::vector<int64_t> vptr(nv + 1, 0);
    for (int64_t i = 0; i < 3 * nt; ++i) ++vptr[T[i] + 1];
    for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int32_t> vtri(3 * nt);
    {
        std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int a = 0; a < 3; ++a) vtri[fill[T[3 * t + a]]++] = int32_t(t);
    }
    std::vector<int32_t> cand;
    for (int64_t t1 = 0; t1 < nt; ++t1) {
        cand.clear();
        for (int a = 0; a < 3; ++a) {
            int32_t v = T[3 * t1 + a];
            for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k)
                if (vtri[k] >= t1) cand.push_back(vtri[k]);
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        const int32_t* a = &T[3 * t1];
        for (int32_t t2 : cand) {
            const int32_t* b = &T[3 * t2];
            int ia[3], ib[3], ns = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    if (a[i] == b[j]) { ia[ns] = i; ib[ns] = j; ++ns; }
            int32_t vs[5] = {-1, -1, -1, -1, -1};
            int8_t type;
            if (ns == 3) {
                type = 3;
                vs[0] = a[0]; vs[1] = a[1]; vs[2] = a[2];
            } else if (ns == 2) {
                type = 2;
                // shared edge A-B in t1's vertex order, then the two opposite vertices
                vs[0] = a[ia[0]]; vs[1] = a[ia[1]];
                vs[2] = a[3 - ia[0] - ia[1]];
                vs[3] = b[3 - ib[0] - ib[1]];
            } else {
                type = 1;
                vs[0] = a[ia[0]];
                vs[1] = a[(ia[0] + 1) % 3]; vs[2] = a[(ia[0] + 2) % 3];
                vs[3] = b[(ib[0] + 1) % 3]; vs[4] = b[(ib[0] + 2) % 3];
            }
            out.t1.push_back(int32_t(t1));
            out.t2.push_back(t2);
            out.type.push_back(type);
            out.verts.insert(out.verts.end(), vs, vs + 5);
            ++out.count[type];
        }
    }
}

// ---- quadrature tables ----------------------------------------------------------------------
void triangle7_rule(double bary[7][3], double w[7]) {
    // Radon's degree-5 rule: centroid (weight 9/40) and the orbits (1-2a, a, a) with
    // a = (6 -+ sqrt 15)/21, weights (155 -+ sqrt 15)/1200; weights sum to 1.
    const double r = std::sqrt(15.0);
    const double a[2] = {(6.0 - r) / 21.0, (6.0 + r) / 21.0};
    const double wa[2] = {(155.0 - r) / 1200.0, (155.0 + r) / 1200.0};
    bary[0][0] = bary[0][1] = bary[0][2] = 1.0 / 3.0;
    w[0] = 9.0 / 40.0;
    int p = 1;
    for (int o = 0; o < 2; ++o)
        for (int k = 0; k < 3; ++k, ++p) {
            for (int c = 0; c < 3; ++c) bary[p][c] = (c == k) ? 1.0 - 2.0 * a[o] : a[o];
            w[p] = wa[o];
        }
}

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
    // roots of P_n by Newton's method from the Chebyshev-like guesses, mapped to [0, 1]
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? z : p1;
            double pm = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // refresh derivative at the converged root
                p0 = 1.0; p1 = z;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1; p1 = p2;
                }
                pn = (n == 1) ? z : p1; pm = (n == 1) ? 1.0 : p0;
                dp = n * (z * pn - pm) / (z * z - 1.0);
                break;
            }
        }
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);   // 2/((1-z^2) P_n'^2) scaled by 1/2
    }
}

}  // namespace bem
