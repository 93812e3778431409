/*
 * Oracle element-pair integrals and Galerkin matrix (TEST INFRASTRUCTURE; see oracle/__init__.py).
 *
 * Plain C, FP64, OpenMP over independent outputs only.  Computes
 *     I(T,T') = 1/(4 pi) * int_T int_T' 1/|x-y| dy dx
 * (the scalar left in Cor. corW once the surface curls, constant on each triangle, are taken out
 * of the integral) and the matrix W_{d,d'} = sum_{T,T'} I(T,T') J_{T,d} . J_{T',d'}.
 *
 * Quadrature (the paper does not fix one; this is the build's reading):
 *   - pairs sharing no vertex: the 7-point degree-5 rule on each triangle (49 evaluations);
 *   - pairs sharing a vertex, an edge, or the whole triangle: Duffy-regularised rules over [0,1]^4
 *     with an n-point Gauss-Legendre rule on every axis.  The regularising maps are derived in
 *     near_* below; they send the singular set to a face of the cube, where their Jacobian
 *     vanishes to the order that cancels 1/|x-y|.
 *
 * Reference triangle: R = {(s,t): 0 <= t <= s <= 1}, chi(s,t) = A + s(B-A) + t(C-B), |det| = 2|T|.
 * Everything here evaluates the kernel at the mapped physical points; no step assumes the kernel
 * is 1/|x-y|, so the same rules integrate the test kernels (1, |x-y|^2, a polynomial) that pin
 * the maps against the product rule.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FOUR_PI 12.566370614359172953850573533118

/* kernel ids: 0 -> 1/|x-y| ; 1 -> 1 ; 2 -> |x-y|^2 ; 3 -> x0*y1 + x2*y2*y0 + x1 (asymmetric) */
static double kern(int id, const double* x, const double* y) {
    double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    switch (id) {
        case 0: return 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        case 1: return 1.0;
        case 2: return d0 * d0 + d1 * d1 + d2 * d2;
        default: return x[0] * y[1] + x[2] * y[2] * y[0] + x[1];
    }
}

static void chi(const double* A, const double* B, const double* C, double s, double t, double* out) {
    for (int k = 0; k < 3; ++k) out[k] = A[k] + s * (B[k] - A[k]) + t * (C[k] - B[k]);
}

static double tri_area(const double* A, const double* B, const double* C) {
    double u[3], v[3], c[3];
    for (int k = 0; k < 3; ++k) { u[k] = B[k] - A[k]; v[k] = C[k] - A[k]; }
    c[0] = u[1] * v[2] - u[2] * v[1];
    c[1] = u[2] * v[0] - u[0] * v[2];
    c[2] = u[0] * v[1] - u[1] * v[0];
    return 0.5 * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
}

/* ---- disjoint pairs: 7 x 7 product rule (bary7: 7x3 barycentric points, w7: weights sum 1) ---- */
double oracle_far_pair(const double* A, const double* B, const double* C,
                       const double* A2, const double* B2, const double* C2,
                       const double* bary7, const double* w7, int kernel) {
    double P[7][3], Q[7][3];
    for (int p = 0; p < 7; ++p)
        for (int k = 0; k < 3; ++k) {
            P[p][k] = bary7[3 * p] * A[k] + bary7[3 * p + 1] * B[k] + bary7[3 * p + 2] * C[k];
            Q[p][k] = bary7[3 * p] * A2[k] + bary7[3 * p + 1] * B2[k] + bary7[3 * p + 2] * C2[k];
        }
    double s = 0.0;
    for (int p = 0; p < 7; ++p)
        for (int q = 0; q < 7; ++q) s += w7[p] * w7[q] * kern(kernel, P[p], Q[q]);
    return s * tri_area(A, B, C) * tri_area(A2, B2, C2) / FOUR_PI;
}

/*
 * Coincident pair, T = T' = (A,B,C).  With z = x^ - y^ the difference body R - R is the hexagon
 * with vertices +-(1,0), +-(1,1), +-(0,1); it is cut into 6 triangles (0, v_i, v_{i+1}) and
 * z = xi * (v_i + eta (v_{i+1} - v_i)).  For fixed z, y^ runs over R n (R - z), which is the copy
 * of R scaled by (1 - xi): in barycentric coordinates beta_k = m_k(z) + (1 - xi) mu_k with
 * m_k(z) = max(0, -L_k(z)), L_k the linear part of the k-th barycentric coordinate
 * (L = (-z1, z1 - z2, z2)), and mu in the unit simplex, mu = (1-m1, m1(1-m2), m1 m2).
 * Jacobian: xi |det(v_i, v_{i+1})| (1 - xi)^2 m1, and |det(v_i, v_{i+1})| = 1 for all six.
 */
static const double HEX[7][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, 0}};

double oracle_near_coincident(const double* A, const double* B, const double* C,
                              int n, const double* gx, const double* gw, int kernel) {
    double sum = 0.0;
    for (int r = 0; r < 6; ++r) {
        for (int a = 0; a < n; ++a) {
            double xi = gx[a];
            for (int b = 0; b < n; ++b) {
                double eta = gx[b];
                double w1 = HEX[r][0] + eta * (HEX[r + 1][0] - HEX[r][0]);
                double w2 = HEX[r][1] + eta * (HEX[r + 1][1] - HEX[r][1]);
                double z1 = xi * w1, z2 = xi * w2;
                double L[3] = {-z1, z1 - z2, z2};
                double m[3];
                for (int k = 0; k < 3; ++k) m[k] = L[k] < 0.0 ? -L[k] : 0.0;
                for (int c = 0; c < n; ++c) {
                    double m1 = gx[c];
                    for (int d = 0; d < n; ++d) {
                        double m2 = gx[d];
                        double mu[3] = {1.0 - m1, m1 * (1.0 - m2), m1 * m2};
                        double beta1 = m[1] + (1.0 - xi) * mu[1];
                        double beta2 = m[2] + (1.0 - xi) * mu[2];
                        double ys = beta1 + beta2, yt = beta2;   /* y^ = beta1 p1 + beta2 p2 */
                        double xs = ys + z1, xt = yt + z2;
                        double x[3], y[3];
                        chi(A, B, C, xs, xt, x);
                        chi(A, B, C, ys, yt, y);
                        double jac = xi * (1.0 - xi) * (1.0 - xi) * m1;
                        sum += gw[a] * gw[b] * gw[c] * gw[d] * jac * kern(kernel, x, y);
                    }
                }
            }
        }
    }
    double ar = tri_area(A, B, C);
    return sum * 4.0 * ar * ar / FOUR_PI;
}

/*
 * Edge pair, T = (A,B,C), T' = (A,B,C'): the common edge is t = t' = 0 in both charts and
 * x - y = (s - s')(B-A) + t (C-B) - t' (C'-B) depends only on w = (s - s', t, t').  For fixed w
 * the anchor s' runs over an interval of length 1 - G(w), G(w) = max(w1,0) + max(w3, w2 - w1).
 * The cone {w2, w3 >= 0} splits into four pieces where G is linear; on each, w = xi * b(eta) with
 * b on the face G = 1 (two square faces, two triangular faces collapsed Duffy-style), and
 * s' = lo(w) + (1 - xi) u.  Jacobian xi^2 (1 - xi) J(eta), J = 1 on the square faces, eta1 on the
 * triangular ones.
 */
double oracle_near_edge(const double* A, const double* B, const double* C, const double* C2,
                        int n, const double* gx, const double* gw, int kernel) {
    double sum = 0.0;
    for (int r = 0; r < 4; ++r)
        for (int a = 0; a < n; ++a) {
            double xi = gx[a];
            for (int b = 0; b < n; ++b) {
                double e1 = gx[b];
                for (int c = 0; c < n; ++c) {
                    double e2 = gx[c];
                    double bb[3], J;
                    int lo_is_w3;
                    switch (r) {
                        case 0: bb[0] = e1; bb[1] = e2; bb[2] = 1.0 - e1; J = 1.0; lo_is_w3 = 1; break;
                        case 1: bb[0] = e1 * (1.0 - e2); bb[1] = 1.0; bb[2] = e1 * e2; J = e1; lo_is_w3 = 0; break;
                        case 2: bb[0] = -e1 * (1.0 - e2); bb[1] = e1 * e2; bb[2] = 1.0; J = e1; lo_is_w3 = 1; break;
                        default: bb[0] = -e1; bb[1] = 1.0 - e1; bb[2] = e2; J = 1.0; lo_is_w3 = 0; break;
                    }
                    double w1 = xi * bb[0], w2 = xi * bb[1], w3 = xi * bb[2];
                    double lo = lo_is_w3 ? w3 : (w2 - w1);
                    for (int d = 0; d < n; ++d) {
                        double u = gx[d];
                        double sp = lo + (1.0 - xi) * u;
                        double s = sp + w1;
                        double x[3], y[3];
                        chi(A, B, C, s, w2, x);
                        chi(A, B, C2, sp, w3, y);
                        double jac = xi * xi * (1.0 - xi) * J;
                        sum += gw[a] * gw[b] * gw[c] * gw[d] * jac * kern(kernel, x, y);
                    }
                }
            }
        }
    return sum * 4.0 * tri_area(A, B, C) * tri_area(A, B, C2) / FOUR_PI;
}

/*
 * Vertex pair, T = (A,B,C), T' = (A,B',C'): the only singular point is s = s' = 0.  Split R x R by
 * which first coordinate is larger; on {s' <= s}: x^ = xi (1, eta1), y^ = xi (eta2, eta2 eta3),
 * and symmetrically on {s <= s'}; Jacobian xi^3 eta2.
 */
double oracle_near_vertex(const double* A, const double* B, const double* C,
                          const double* B2, const double* C2,
                          int n, const double* gx, const double* gw, int kernel) {
    double sum = 0.0;
    for (int r = 0; r < 2; ++r)
        for (int a = 0; a < n; ++a) {
            double xi = gx[a];
            for (int b = 0; b < n; ++b)
                for (int c = 0; c < n; ++c)
                    for (int d = 0; d < n; ++d) {
                        double e1 = gx[b], e2 = gx[c], e3 = gx[d];
                        double ps = xi, pt = xi * e1, qs = xi * e2, qt = xi * e2 * e3;
                        double x[3], y[3];
                        if (r == 0) {
                            chi(A, B, C, ps, pt, x);
                            chi(A, B2, C2, qs, qt, y);
                        } else {
                            chi(A, B, C, qs, qt, x);
                            chi(A, B2, C2, ps, pt, y);
                        }
                        double jac = xi * xi * xi * e2;
                        sum += gw[a] * gw[b] * gw[c] * gw[d] * jac * kern(kernel, x, y);
                    }
        }
    return sum * 4.0 * tri_area(A, B, C) * tri_area(A, B2, C2) / FOUR_PI;
}

/* ---- classification by shared vertex indices and the pair integral ---------------------- */
typedef struct {
    const double* V;
    const int32_t* T;
    const double* bary7;
    const double* w7;
    int n;
    const double* gx;
    const double* gw;
} ctx_t;

static double pair_integral(const ctx_t* c, int t1, int t2) {
    if (t1 > t2) { int tmp = t1; t1 = t2; t2 = tmp; }  /* symmetric by construction */
    const int32_t* a = c->T + 3 * t1;
    const int32_t* b = c->T + 3 * t2;
    int shared = 0, ia[3], ib[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (a[i] == b[j]) { ia[shared] = i; ib[shared] = j; ++shared; }
#define VX(k) (c->V + 3 * (size_t)(k))
    if (shared == 0)
        return oracle_far_pair(VX(a[0]), VX(a[1]), VX(a[2]), VX(b[0]), VX(b[1]), VX(b[2]),
                               c->bary7, c->w7, 0);
    if (shared == 3)
        return oracle_near_coincident(VX(a[0]), VX(a[1]), VX(a[2]), c->n, c->gx, c->gw, 0);
    if (shared == 2) {
        int P = a[ia[0]], Q = a[ia[1]];
        int R1 = a[3 - ia[0] - ia[1]], R2 = b[3 - ib[0] - ib[1]];
        return oracle_near_edge(VX(P), VX(Q), VX(R1), VX(R2), c->n, c->gx, c->gw, 0);
    }
    /* one shared vertex: put it first, keep the others in cyclic order */
    int P = a[ia[0]];
    int B1 = a[(ia[0] + 1) % 3], C1 = a[(ia[0] + 2) % 3];
    int B2 = b[(ib[0] + 1) % 3], C2 = b[(ib[0] + 2) % 3];
    return oracle_near_vertex(VX(P), VX(B1), VX(C1), VX(B2), VX(C2), c->n, c->gx, c->gw, 0);
#undef VX
}

void oracle_pair_integrals(const double* V, const int32_t* T, const double* bary7, const double* w7,
                           int n, const double* gx, const double* gw,
                           int64_t npairs, const int32_t* pairs, double* out) {
    ctx_t c = {V, T, bary7, w7, n, gx, gw};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < npairs; ++p) out[p] = pair_integral(&c, pairs[2 * p], pairs[2 * p + 1]);
}

/* rows r0 .. r0+nrows-1 of the full N_T x N_T matrix I */
void oracle_I_rows(const double* V, const int32_t* T, int64_t nt, const double* bary7, const double* w7,
                   int n, const double* gx, const double* gw, int64_t r0, int64_t nrows, double* out) {
    ctx_t c = {V, T, bary7, w7, n, gx, gw};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t t2 = 0; t2 < nt; ++t2) out[r * nt + t2] = pair_integral(&c, (int)(r0 + r), (int)t2);
}

/*
 * Contraction of one panel of rows of I (triangles r0 .. r0+nr-1, rows of length nt) into rows
 * d0 .. d1-1 of W: for every dof d in that range, the triangles of its star that fall in the panel
 * contribute
 *     Wout[d - d0][d2] += I(T1,T2) * (J_{T1,d} . J_{T2,d2})   for d2 >= d.
 * Wout has (d1 - d0) rows of N.
 */
void oracle_W_accumulate(int64_t nt, int64_t N, const int64_t* tri_ptr, const int64_t* tri_dof,
                         const double* tri_J, const int64_t* dof_ptr, const int64_t* dof_tri,
                         const double* dof_J, int64_t r0, int64_t nr, const double* I, int64_t d0,
                         int64_t d1, double* Wout) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t d = d0; d < d1; ++d) {
        double* Wd = Wout + (d - d0) * N;
        for (int64_t e = dof_ptr[d]; e < dof_ptr[d + 1]; ++e) {
            int64_t t1 = dof_tri[e];
            if (t1 < r0 || t1 >= r0 + nr) continue;
            const double* J1 = dof_J + 3 * e;
            const double* Irow = I + (t1 - r0) * nt;
            for (int64_t t2 = 0; t2 < nt; ++t2) {
                double iv = Irow[t2];
                for (int64_t f = tri_ptr[t2]; f < tri_ptr[t2 + 1]; ++f) {
                    int64_t d2 = tri_dof[f];
                    if (d2 < d) continue;
                    const double* J2 = tri_J + 3 * f;
                    Wd[d2] += iv * (J1[0] * J2[0] + J1[1] * J2[1] + J1[2] * J2[2]);
                }
            }
        }
    }
}

/*
 * Full W (N x N, row-major).  I is produced in panels of triangle rows and each panel is
 * contracted into W (oracle_W_accumulate, upper triangle d2 >= d); the strict lower triangle is
 * mirrored at the end, so W is exactly symmetric.
 * tri_ptr/tri_dof/tri_J: CSR triangle -> (dof, J); dof_ptr/dof_tri/dof_J: CSR dof -> (triangle, J).
 */
void oracle_W(const double* V, const int32_t* T, int64_t nt, const double* bary7, const double* w7,
              int n, const double* gx, const double* gw, int64_t N,
              const int64_t* tri_ptr, const int64_t* tri_dof, const double* tri_J,
              const int64_t* dof_ptr, const int64_t* dof_tri, const double* dof_J,
              int64_t panel, double* W) {
    memset(W, 0, sizeof(double) * (size_t)N * (size_t)N);
    double* I = (double*)malloc(sizeof(double) * (size_t)panel * (size_t)nt);
    for (int64_t r0 = 0; r0 < nt; r0 += panel) {
        int64_t nr = (r0 + panel <= nt) ? panel : nt - r0;
        oracle_I_rows(V, T, nt, bary7, w7, n, gx, gw, r0, nr, I);
        oracle_W_accumulate(nt, N, tri_ptr, tri_dof, tri_J, dof_ptr, dof_tri, dof_J, r0, nr, I, 0, N, W);
    }
    free(I);
    for (int64_t d = 0; d < N; ++d)
        for (int64_t d2 = 0; d2 < d; ++d2) W[d * N + d2] = W[d2 * N + d];
}

/* selected rows of W: out[k][:] = W[rows[k]][:] computed directly from its star */
void oracle_W_rows(const double* V, const int32_t* T, int64_t nt, const double* bary7, const double* w7,
                   int n, const double* gx, const double* gw, int64_t N,
                   const int64_t* tri_ptr, const int64_t* tri_dof, const double* tri_J,
                   const int64_t* dof_ptr, const int64_t* dof_tri, const double* dof_J,
                   int64_t nrows, const int64_t* rows, double* out) {
    ctx_t c = {V, T, bary7, w7, n, gx, gw};
    memset(out, 0, sizeof(double) * (size_t)nrows * (size_t)N);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t d = rows[k];
        double* o = out + k * N;
        for (int64_t e = dof_ptr[d]; e < dof_ptr[d + 1]; ++e) {
            int t1 = (int)dof_tri[e];
            const double* J1 = dof_J + 3 * e;
            for (int64_t t2 = 0; t2 < nt; ++t2) {
                double iv = pair_integral(&c, t1, (int)t2);
                for (int64_t f = tri_ptr[t2]; f < tri_ptr[t2 + 1]; ++f) {
                    const double* J2 = tri_J + 3 * f;
                    o[tri_dof[f]] += iv * (J1[0] * J2[0] + J1[1] * J2[1] + J1[2] * J2[2]);
                }
            }
        }
    }
}

/* generic near-rule entry for the pins: type 3 coincident, 2 edge, 1 vertex; P = 6 or 9 doubles */
double oracle_near_generic(int type, const double* X, const double* Y, int n, const double* gx,
                           const double* gw, int kernel) {
    if (type == 3) return oracle_near_coincident(X, X + 3, X + 6, n, gx, gw, kernel);
    if (type == 2) return oracle_near_edge(X, X + 3, X + 6, Y + 6, n, gx, gw, kernel);
    return oracle_near_vertex(X, X + 3, X + 6, Y + 3, Y + 6, n, gx, gw, kernel);
}
