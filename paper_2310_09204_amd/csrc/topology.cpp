// Host-side analysis of a polygonal multiscreen mesh: validation, generalized vertices
// (sectors), jump-basis degrees of freedom, jump coefficients and the near-pair list.
//
// Paper, Section 4.2: around vertex x_i the complement of Gamma splits into q_i connected sectors
// (components of the star graph G(x_i), eqs. defCurlyHOmega/defCurlyHGamma).  The jump basis is
// psi_{i,j} = phi_{i,j} - phi_{i,q_i}, j < q_i (eqs. defCurlyHtildeGamma, defYij).  Section 4.3
// evaluates everything on oriented triangles (T, side); which sides share a sector at a vertex
// is what the sets alpha_{k,l} (eq. defAlphaij) record.
//
// Surface-only construction used here, vertex by vertex (vertices are independent, so they are
// processed on a few host threads): the sides (T, +/-) of the triangles of the vertex star are the
// nodes of a small union-find.  Around each edge at the vertex the incident triangles are ordered
// by angle; the side of a triangle facing the next triangle is merged with that triangle's side
// facing back; at a free edge the two sides of its triangle are merged.  The classes are the
// sectors.  Because the union keeps the smaller node as root and the star lists triangles in
// increasing index order, each root is the sector's (triangle index, + before -) first side,
// which is the canonical label order.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <thread>

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

// index of (triangle, corner, side) in the per-mesh sector table
inline int64_t side_node(int64_t t, int a, int s) { return (t * 3 + a) * 2 + s; }

}  // namespace

void analyze_mesh(const double* Vin, int64_t nv, const int32_t* Tin, int64_t nt, MeshTopo& m, const int32_t* tri_user,
                  const int32_t* vert_user) {
    if (!Vin || !Tin || nv <= 0 || nt <= 0) fail(BEM_E_INVALID_ARG, "empty mesh");
    // indices as the caller numbered them (messages, and the order that labels sectors)
    auto tu = [&](int64_t t) { return std::to_string(tri_user ? int64_t(tri_user[t]) : t); };
    auto vu = [&](int64_t v) { return std::to_string(vert_user ? int64_t(vert_user[v]) : v); };
    auto ukey_v = [&](int64_t v) { return vert_user ? int64_t(vert_user[v]) : v; };
    auto ukey_t = [&](int64_t t) { return tri_user ? int64_t(tri_user[t]) : t; };
    if (nt > (int64_t(1) << 30)) fail(BEM_E_INVALID_ARG, "too many triangles");
    m = MeshTopo();
    m.nv = nv;
    m.nt = nt;
    m.V.assign(Vin, Vin + 3 * nv);
    m.T.assign(Tin, Tin + 3 * nt);
    const auto& V = m.V;
    const auto& T = m.T;

    // indices and coordinates, then element geometry, on threads; the error reported is the one of
    // the first failing triangle, as in a sequential pass
    m.normal.resize(3 * nt);
    m.area.resize(nt);
    {
        FirstFailure bad;
        parallel_for(nt, [&](int64_t tb, int64_t te) {
            for (int64_t t = tb; t < te; ++t) {
                try {
                    for (int a = 0; a < 3; ++a) {
                        int32_t v = T[3 * t + a];
                        if (v < 0 || v >= nv) fail(BEM_E_INVALID_ARG, "triangle " + tu(t) + " has a vertex index out of range");
                        if (!std::isfinite(V[3 * v]) || !std::isfinite(V[3 * v + 1]) || !std::isfinite(V[3 * v + 2]))
                            fail(BEM_E_INVALID_ARG, "non-finite vertex coordinate");
                    }
                    if (T[3 * t] == T[3 * t + 1] || T[3 * t + 1] == T[3 * t + 2] || T[3 * t] == T[3 * t + 2])
                        fail(BEM_E_DEGENERATE, "triangle " + tu(t) + " repeats a vertex");
                } catch (const Failure& f) {
                    bad.record(ukey_t(t), f);
                    return;
                }
            }
        });
        bad.rethrow();
    }

    // ---- element geometry --------------------------------------------------------------------
    {
        FirstFailure bad;
        parallel_for(nt, [&](int64_t tb, int64_t te) {
            for (int64_t t = tb; t < te; ++t) {
                Vec3 x0 = at(V, T[3 * t]), x1 = at(V, T[3 * t + 1]), x2 = at(V, T[3 * t + 2]);
                Vec3 e1 = minus(x1, x0), e2 = minus(x2, x0), e3 = minus(x2, x1);
                Vec3 c = cross3(e1, e2);
                double tw = norm3(c);
                double scale = std::max({dot3(e1, e1), dot3(e2, e2), dot3(e3, e3)});
                if (!(tw > 1e-12 * scale)) {
                    bad.record(ukey_t(t), Failure{BEM_E_DEGENERATE, "triangle " + tu(t) + " has zero area"});
                    return;
                }
                for (int k = 0; k < 3; ++k) m.normal[3 * t + k] = c[k] / tw;
                m.area[t] = 0.5 * tw;
            }
        });
        bad.rethrow();
    }

    // ---- repeated vertices (by coordinates) ------------------------------------------------------
    {
        std::vector<char> used(nv, 0);
        for (int64_t i = 0; i < 3 * nt; ++i) used[T[i]] = 1;
        std::vector<int64_t> order;
        for (int64_t v = 0; v < nv; ++v) if (used[v]) order.push_back(v);
        auto less = [&](int64_t a, int64_t b) {
            for (int k = 0; k < 3; ++k)
                if (V[3 * a + k] != V[3 * b + k]) return V[3 * a + k] < V[3 * b + k];
            return a < b;
        };
        // (coordinates, index) is a strict total order
        parallel_sort(order.begin(), int64_t(order.size()), less);
        for (size_t i = 1; i < order.size(); ++i) {
            int64_t a = order[i - 1], b = order[i];
            if (V[3 * a] == V[3 * b] && V[3 * a + 1] == V[3 * b + 1] && V[3 * a + 2] == V[3 * b + 2])
                fail(BEM_E_MESH_NONCONFORMING, "vertices " + vu(a) + " and " + vu(b) + " coincide");
        }
    }

    // ---- vertex stars (counting sort; triangles of a star in increasing index order, the
    //      caller's numbering when tri_user is given) ---------------------------------------------
    std::vector<int64_t> vptr(nv + 1, 0);
    for (int64_t i = 0; i < 3 * nt; ++i) ++vptr[T[i] + 1];
    for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int32_t> vtri(3 * nt);
    {
        std::vector<int32_t> by_user;
        if (tri_user) {
            by_user.resize(size_t(nt));
            for (int64_t t = 0; t < nt; ++t) by_user[size_t(tri_user[t])] = int32_t(t);
        }
        std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t u = 0; u < nt; ++u) {
            const int64_t t = tri_user ? by_user[size_t(u)] : u;
            for (int a = 0; a < 3; ++a) vtri[fill[T[3 * t + a]]++] = int32_t(t);
        }
    }
    auto corner_of = [&](int64_t t, int64_t v) -> int {
        for (int a = 0; a < 3; ++a) if (T[3 * t + a] == v) return a;
        return -1;
    };

    // ---- sectors, vertex by vertex (independent: only the fans of the vertex's own edges matter) --
    m.q.assign(nv, 0);
    m.sector.assign(6 * nt, -1);
    FirstFailure err;
    parallel_for(nv, [&](int64_t vb, int64_t ve) {
        struct EdgeEnd { int32_t w; int32_t lt; };
        struct Item { double theta; int32_t lt; Vec3 d; };
        std::vector<EdgeEnd> ends;
        std::vector<Item> fan;
        std::vector<int64_t> roots;
        std::vector<std::array<int32_t, 2>> pairs;
        for (int64_t v = vb; v < ve; ++v) {
            const int64_t s0 = vptr[v], ns = vptr[v + 1] - s0;
            if (ns == 0) continue;
            try {
                // repeated triangles meet at their smallest vertex with the same other two vertices
                pairs.clear();
                for (int64_t k = 0; k < ns; ++k) {
                    const int64_t t = vtri[s0 + k];
                    int32_t o[2], c = 0;
                    for (int a = 0; a < 3; ++a) if (T[3 * t + a] != v) o[c++] = T[3 * t + a];
                    if (o[0] > o[1]) std::swap(o[0], o[1]);
                    pairs.push_back({o[0], o[1]});
                }
                {
                    auto sp = pairs;
                    std::sort(sp.begin(), sp.end());
                    for (size_t k = 1; k < sp.size(); ++k)
                        if (sp[k] == sp[k - 1]) fail(BEM_E_MESH_NONCONFORMING, "repeated triangle");
                }
                ends.clear();
                for (int64_t k = 0; k < ns; ++k) {
                    ends.push_back({pairs[k][0], int32_t(k)});
                    ends.push_back({pairs[k][1], int32_t(k)});
                }
                std::sort(ends.begin(), ends.end(), [](const EdgeEnd& x, const EdgeEnd& y) {
                    return x.w != y.w ? x.w < y.w : x.lt < y.lt;
                });
                DisjointSets sides(2 * ns), tris(ns);
                for (size_t b = 0; b < ends.size();) {
                    size_t e = b;
                    while (e < ends.size() && ends[e].w == ends[b].w) ++e;
                    const int64_t w = ends[b].w;
                    for (size_t k = b + 1; k < e; ++k) tris.join(ends[b].lt, ends[k].lt);
                    if (e - b == 1) {
                        sides.join(2 * ends[b].lt, 2 * ends[b].lt + 1);
                    } else {
                        Vec3 axis = minus(at(V, w), at(V, v));
                        const double al = norm3(axis);
                        for (auto& c : axis) c /= al;
                        fan.clear();
                        for (size_t k = b; k < e; ++k) {
                            const int64_t t = vtri[s0 + ends[k].lt];
                            const int64_t third = int64_t(T[3 * t]) + T[3 * t + 1] + T[3 * t + 2] - v - w;
                            Vec3 d = minus(at(V, third), at(V, v));
                            const double along = dot3(d, axis);
                            for (int c = 0; c < 3; ++c) d[c] -= along * axis[c];
                            const double dn = norm3(d);
                            for (auto& c : d) c /= dn;
                            fan.push_back({0.0, ends[k].lt, d});
                        }
                        const Vec3 b1 = fan[0].d;
                        const Vec3 b2 = cross3(axis, b1);
                        for (auto& it : fan) {
                            const double th = std::atan2(dot3(it.d, b2), dot3(it.d, b1));
                            it.theta = th < 0 ? th + 2.0 * M_PI : th;
                        }
                        std::sort(fan.begin(), fan.end(), [](const Item& x, const Item& y) { return x.theta < y.theta; });
                        const size_t nf = fan.size();
                        for (size_t k = 0; k < nf; ++k) {
                            const double gap = (k + 1 < nf) ? fan[k + 1].theta - fan[k].theta : fan[0].theta + 2.0 * M_PI - fan[k].theta;
                            if (gap < 1e-9)
                                fail(BEM_E_MESH_NONCONFORMING, "two triangles at edge (" +
                                                                   std::to_string(std::min(ukey_v(v), ukey_v(w))) + "," +
                                                                   std::to_string(std::max(ukey_v(v), ukey_v(w))) +
                                                                   ") lie in the same half-plane");
                        }
                        for (size_t k = 0; k < nf; ++k) {
                            const Item& A = fan[k];
                            const Item& B = fan[(k + 1) % nf];
                            const int64_t ta = vtri[s0 + A.lt], tb = vtri[s0 + B.lt];
                            // side facing increasing angle: '+' (0) iff n_T . (axis x d_T) > 0
                            const Vec3 na = {m.normal[3 * ta], m.normal[3 * ta + 1], m.normal[3 * ta + 2]};
                            const Vec3 nb = {m.normal[3 * tb], m.normal[3 * tb + 1], m.normal[3 * tb + 2]};
                            const int inc_a = dot3(na, cross3(axis, A.d)) > 0 ? 0 : 1;
                            const int inc_b = dot3(nb, cross3(axis, B.d)) > 0 ? 0 : 1;
                            sides.join(2 * A.lt + inc_a, 2 * B.lt + (1 - inc_b));
                        }
                    }
                    b = e;
                }
                for (int64_t k = 1; k < ns; ++k)
                    if (tris.root(k) != tris.root(0)) fail(BEM_E_POINT_CONTACT, "point contact at vertex " + vu(v));
                // sectors labelled by their smallest member (local order = the star's triangle order)
                roots.clear();
                for (int64_t k = 0; k < 2 * ns; ++k) roots.push_back(sides.root(k));
                std::sort(roots.begin(), roots.end());
                roots.erase(std::unique(roots.begin(), roots.end()), roots.end());
                m.q[v] = int32_t(roots.size());
                for (int64_t k = 0; k < ns; ++k) {
                    const int64_t t = vtri[s0 + k];
                    const int a = corner_of(t, v);
                    for (int sd = 0; sd < 2; ++sd)
                        m.sector[side_node(t, a, sd)] =
                            int32_t(std::lower_bound(roots.begin(), roots.end(), sides.root(2 * k + sd)) - roots.begin());
                }
            } catch (const Failure& f) {
                err.record(ukey_v(v), f);
            }
        }
    });
    err.rethrow();

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
    auto coeff = [&](int64_t t, int a, int32_t j) {
        const int32_t qv = m.q[T[3 * t + a]];
        const int32_t sp = m.sector[side_node(t, a, 0)], sm = m.sector[side_node(t, a, 1)];
        return ((sp == j) ? 1 : (sp == qv - 1 ? -1 : 0)) - ((sm == j) ? 1 : (sm == qv - 1 ? -1 : 0));
    };
    m.tri_ptr.assign(nt + 1, 0);
    parallel_for(nt, [&](int64_t tb, int64_t te) {
        for (int64_t t = tb; t < te; ++t) {
            int64_t cnt = 0;
            for (int a = 0; a < 3; ++a)
                for (int32_t j = 0; j + 1 < m.q[T[3 * t + a]]; ++j) cnt += coeff(t, a, j) != 0;
            m.tri_ptr[t + 1] = cnt;
        }
    });
    for (int64_t t = 0; t < nt; ++t) m.tri_ptr[t + 1] += m.tri_ptr[t];
    const int64_t ne = m.tri_ptr[nt];
    m.tri_dof.resize(ne); m.tri_corner.resize(ne); m.tri_c.resize(ne);
    parallel_for(nt, [&](int64_t tb, int64_t te) {
        for (int64_t t = tb; t < te; ++t) {
            int64_t pos = m.tri_ptr[t];
            for (int a = 0; a < 3; ++a) {
                const int32_t v = T[3 * t + a];
                for (int32_t j = 0; j + 1 < m.q[v]; ++j) {
                    const int c = coeff(t, a, j);
                    if (c == 0) continue;
                    m.tri_dof[pos] = int32_t(m.first_dof[v] + j);
                    m.tri_corner[pos] = int8_t(a);
                    m.tri_c[pos] = int8_t(c);
                    ++pos;
                }
            }
        }
    });
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

void analyze_segments(const double* Vin, int64_t nv, const int32_t* Sin, int64_t ns, MeshTopo& m) {
    if (!Vin || !Sin || nv <= 0 || ns <= 0) fail(BEM_E_INVALID_ARG, "empty mesh");
    if (ns > (int64_t(1) << 30)) fail(BEM_E_INVALID_ARG, "too many segments");
    m = MeshTopo();
    m.dim = 2;
    m.nv = nv;
    m.nt = ns;
    m.V.assign(size_t(nv) * 3, 0.0);
    for (int64_t v = 0; v < nv; ++v) {
        if (!std::isfinite(Vin[2 * v]) || !std::isfinite(Vin[2 * v + 1])) fail(BEM_E_INVALID_ARG, "non-finite vertex coordinate");
        m.V[3 * v] = Vin[2 * v];
        m.V[3 * v + 1] = Vin[2 * v + 1];
    }
    m.S.assign(Sin, Sin + 2 * ns);
    m.normal.assign(size_t(ns) * 3, 0.0);
    m.area.assign(size_t(ns), 0.0);
    double extent = 0.0;
    for (int64_t i = 0; i < 2 * nv; ++i) extent = std::max(extent, std::fabs(Vin[i]));
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t a = Sin[2 * s], b = Sin[2 * s + 1];
        if (a < 0 || a >= nv || b < 0 || b >= nv) fail(BEM_E_INVALID_ARG, "segment " + std::to_string(s) + " has a vertex index out of range");
        const double dx = Vin[2 * b] - Vin[2 * a], dy = Vin[2 * b + 1] - Vin[2 * a + 1];
        const double len = std::sqrt(dx * dx + dy * dy);
        if (a == b || !(len > 1e-12 * std::max(extent, 1e-300))) fail(BEM_E_DEGENERATE, "segment " + std::to_string(s) + " has zero length");
        m.area[s] = len;
        m.normal[3 * s] = -dy / len;
        m.normal[3 * s + 1] = dx / len;
    }
    // incident segment ends per vertex, sorted by the angle of the direction leaving the vertex
    std::vector<int64_t> vptr(nv + 1, 0);
    for (int64_t i = 0; i < 2 * ns; ++i) ++vptr[Sin[i] + 1];
    for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int64_t> ends(2 * ns);   // 2 s + a
    {
        std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t s = 0; s < ns; ++s)
            for (int a = 0; a < 2; ++a) ends[fill[Sin[2 * s + a]]++] = 2 * s + a;
    }
    // sector label of side (s, end a, side sd): index [4 s + 2 a + sd], sd 0 = side +, 1 = side -
    m.sector.assign(size_t(ns) * 4, -1);
    m.q.assign(nv, 0);
    for (int64_t v = 0; v < nv; ++v) {
        const int64_t deg = vptr[v + 1] - vptr[v];
        if (deg == 0) continue;
        std::vector<std::pair<double, int64_t>> dir;
        for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
            const int64_t s = ends[k] / 2;
            const int a = int(ends[k] % 2);
            const int32_t o = Sin[2 * s + 1 - a];   // the other end
            dir.emplace_back(std::atan2(Vin[2 * o + 1] - Vin[2 * v + 1], Vin[2 * o] - Vin[2 * v]), ends[k]);
        }
        std::sort(dir.begin(), dir.end());
        for (size_t k = 0; k + 1 < dir.size(); ++k)
            if (dir[k + 1].first - dir[k].first < 1e-9) {
                const int64_t s1 = dir[k].second / 2, s2 = dir[k + 1].second / 2;
                fail(BEM_E_MESH_NONCONFORMING, s1 == s2 ? "repeated segment" :
                     "segments " + std::to_string(s1) + " and " + std::to_string(s2) + " overlap at vertex " + std::to_string(v));
            }
        // sector k: the counter-clockwise hand of direction k and the clockwise hand of direction
        // k + 1.  Leaving v along segment s, the counter-clockwise hand is side + if s starts at v
        // (n_s is tau_s turned counter-clockwise) and side - if it ends there.
        const int64_t mdeg = int64_t(dir.size());
        std::vector<std::array<int64_t, 2>> mem(mdeg);   // members as 2 s + side
        for (int64_t k = 0; k < mdeg; ++k) {
            const int64_t e1 = dir[k].second, e2 = dir[(k + 1) % mdeg].second;
            const int64_t ccw = 2 * (e1 / 2) + ((e1 % 2 == 0) ? 0 : 1);
            const int64_t cw = 2 * (e2 / 2) + ((e2 % 2 == 0) ? 1 : 0);
            mem[k] = {std::min(ccw, cw), std::max(ccw, cw)};
        }
        std::vector<int64_t> order(mdeg);
        for (int64_t k = 0; k < mdeg; ++k) order[k] = k;
        std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return mem[x][0] < mem[y][0]; });
        for (int64_t lab = 0; lab < mdeg; ++lab)
            for (int64_t node : mem[order[lab]]) {
                const int64_t s = node / 2;
                const int sd = int(node % 2);
                const int a = (Sin[2 * s] == v) ? 0 : 1;
                m.sector[4 * s + 2 * a + sd] = int32_t(lab);
            }
        m.q[v] = int32_t(mdeg);
    }
    // dofs and jump coefficients, as for triangles
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
    auto coeff = [&](int64_t s, int a, int32_t j) {
        const int32_t qv = m.q[Sin[2 * s + a]];
        const int32_t sp = m.sector[4 * s + 2 * a], sm = m.sector[4 * s + 2 * a + 1];
        return ((sp == j) ? 1 : (sp == qv - 1 ? -1 : 0)) - ((sm == j) ? 1 : (sm == qv - 1 ? -1 : 0));
    };
    m.tri_ptr.assign(ns + 1, 0);
    for (int64_t s = 0; s < ns; ++s) {
        int64_t cnt = 0;
        for (int a = 0; a < 2; ++a)
            for (int32_t j = 0; j + 1 < m.q[Sin[2 * s + a]]; ++j) cnt += coeff(s, a, j) != 0;
        m.tri_ptr[s + 1] = m.tri_ptr[s] + cnt;
    }
    const int64_t ne = m.tri_ptr[ns];
    m.tri_dof.resize(ne); m.tri_corner.resize(ne); m.tri_c.resize(ne);
    for (int64_t s = 0; s < ns; ++s) {
        int64_t pos = m.tri_ptr[s];
        for (int a = 0; a < 2; ++a) {
            const int32_t v = Sin[2 * s + a];
            for (int32_t j = 0; j + 1 < m.q[v]; ++j) {
                const int c = coeff(s, a, j);
                if (c == 0) continue;
                m.tri_dof[pos] = int32_t(m.first_dof[v] + j);
                m.tri_corner[pos] = int8_t(a);
                m.tri_c[pos] = int8_t(c);
                ++pos;
            }
        }
    }
    m.dof_ptr.assign(m.N + 1, 0);
    for (int64_t e = 0; e < ne; ++e) ++m.dof_ptr[m.tri_dof[e] + 1];
    for (int64_t d = 0; d < m.N; ++d) m.dof_ptr[d + 1] += m.dof_ptr[d];
    m.dof_tri.resize(ne); m.dof_corner.resize(ne); m.dof_c.resize(ne);
    std::vector<int64_t> fill(m.dof_ptr.begin(), m.dof_ptr.end() - 1);
    for (int64_t s = 0; s < ns; ++s)
        for (int64_t e = m.tri_ptr[s]; e < m.tri_ptr[s + 1]; ++e) {
            const int64_t pos = fill[m.tri_dof[e]]++;
            m.dof_tri[pos] = int32_t(s);
            m.dof_corner[pos] = m.tri_corner[e];
            m.dof_c[pos] = m.tri_c[e];
        }
}

// Morton code of a point quantised to 21 bits per axis: the bits of x, y and z interleaved
static uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    auto spread = [](uint64_t v) {
        v &= 0x1fffff;
        v = (v | (v << 32)) & 0x1f00000000ffffull;
        v = (v | (v << 16)) & 0x1f0000ff0000ffull;
        v = (v | (v << 8)) & 0x100f00f00f00f00full;
        v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
        v = (v | (v << 2)) & 0x1249249249249249ull;
        return v;
    };
    return spread(x) | (spread(y) << 1) | (spread(z) << 2);
}

void locality_order(const double* V, int64_t nv, const int32_t* T, int64_t nt, std::vector<int32_t>& vert_user,
                    std::vector<int32_t>& tri_user) {
    double lo[3] = {V[0], V[1], V[2]}, hi[3] = {V[0], V[1], V[2]};
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], V[3 * i + c]);
            hi[c] = std::max(hi[c], V[3 * i + c]);
        }
    const double span = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    auto key = [&](double x, double y, double z) {
        auto q = [&](double v, int c) {
            const double f = (v - lo[c]) / span;
            return uint32_t(std::min(2097151.0, std::max(0.0, f * 2097151.0)));
        };
        return morton3(q(x, 0), q(y, 1), q(z, 2));
    };
    std::vector<std::pair<uint64_t, int32_t>> kv(static_cast<size_t>(nv)), kt(static_cast<size_t>(nt));
    parallel_for(nv, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) kv[size_t(i)] = {key(V[3 * i], V[3 * i + 1], V[3 * i + 2]), int32_t(i)};
    });
    parallel_for(nt, [&](int64_t b, int64_t e) {
        for (int64_t t = b; t < e; ++t) {
            double c[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < 3; ++k) c[k] += V[3 * int64_t(T[3 * t + a]) + k] / 3.0;
            kt[size_t(t)] = {key(c[0], c[1], c[2]), int32_t(t)};
        }
    });
    // (key, index) pairs: a strict total order
    parallel_sort(kv.begin(), nv, std::less<std::pair<uint64_t, int32_t>>());
    parallel_sort(kt.begin(), nt, std::less<std::pair<uint64_t, int32_t>>());
    vert_user.resize(size_t(nv));
    tri_user.resize(size_t(nt));
    for (int64_t i = 0; i < nv; ++i) vert_user[size_t(i)] = kv[size_t(i)].second;
    for (int64_t t = 0; t < nt; ++t) tri_user[size_t(t)] = kt[size_t(t)].second;
}

void build_near_list(const MeshTopo& m, NearList& out, const int32_t* tri_user) {
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
    // triangles in chunks of 2048; each chunk fills its own list, joined in chunk order
    const int64_t csz = 2048;
    const int64_t nchunk = (nt + csz - 1) / csz;
    std::vector<NearList> parts(nchunk);
    parallel_for(nt, [&](int64_t tb, int64_t te) {
        std::vector<int32_t> cand;
        for (int64_t c = (tb + csz - 1) / csz; c * csz < te; ++c) {
            NearList& o = parts[c];
            for (int64_t t1 = c * csz; t1 < std::min(nt, (c + 1) * csz); ++t1) {
                cand.clear();
                for (int a = 0; a < 3; ++a) {
                    const int32_t v = T[3 * t1 + a];
                    for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k)
                        if (vtri[k] >= t1) cand.push_back(vtri[k]);
                }
                std::sort(cand.begin(), cand.end());
                cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
                for (int32_t t2c : cand) {
                    // the pair's first triangle is the one with the smaller index in the caller's
                    // numbering: the Duffy rules are not symmetric in the two triangles, and this is
                    // the order in which the unrenumbered problem (and the oracle) takes them
                    int32_t f = int32_t(t1), t2 = t2c;
                    if (tri_user && tri_user[t2] < tri_user[f]) std::swap(f, t2);
                    const int32_t* a = &T[3 * int64_t(f)];
                    const int32_t* b = &T[3 * int64_t(t2)];
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
                    o.t1.push_back(f);
                    o.t2.push_back(t2);
                    o.type.push_back(type);
                    o.verts.insert(o.verts.end(), vs, vs + 5);
                    ++o.count[type];
                }
            }
        }
    });
    // join in chunk order: offsets first, then the copies in parallel
    std::vector<size_t> off(parts.size() + 1, 0);
    for (size_t c = 0; c < parts.size(); ++c) {
        off[c + 1] = off[c] + parts[c].t1.size();
        for (int k = 0; k < 4; ++k) out.count[k] += parts[c].count[k];
    }
    const size_t total = off.back();
    out.t1.resize(total);
    out.t2.resize(total);
    out.type.resize(total);
    out.verts.resize(5 * total);
    parallel_for(int64_t(parts.size()), [&](int64_t cb, int64_t ce) {
        for (int64_t c = cb; c < ce; ++c) {
            const NearList& o = parts[size_t(c)];
            const size_t b = off[size_t(c)];
            std::copy(o.t1.begin(), o.t1.end(), out.t1.begin() + b);
            std::copy(o.t2.begin(), o.t2.end(), out.t2.begin() + b);
            std::copy(o.type.begin(), o.type.end(), out.type.begin() + b);
            std::copy(o.verts.begin(), o.verts.end(), out.verts.begin() + 5 * b);
        }
    }, 1);
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
