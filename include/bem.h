/*
 * bem.h - C-ABI of the MI355X hypersingular BEM library (libbem.so).
 *
 * Problem (Averseng, Claeys, Hiptmair, "Boundary Element Methods for the Laplace Hypersingular
 * Integral Equation on Multiscreens: a two-level Substructuring Preconditioner"):
 *   the exterior Laplace Neumann problem on a polygonal multiscreen Gamma (eq. PDE_intro,
 *   Def. polygonalMS) is solved as U = DL(phi) with phi in the jump space H~^{1/2}([Gamma])
 *   satisfying a(phi, psi) = l_g(psi) (Thm. thmBVP).  Its Galerkin discretisation on the
 *   conforming space V~_h([Gamma]) of jumps of piecewise-linear functions (Section 4.2) is the
 *   dense symmetric positive definite system  W Phi = L  (Section 4.1).
 *
 * Conventions shared by every call
 *   - Meshes: vertices double[nv][3]; triangles int32[nt][3] (vertex order fixes n_T =
 *     (x1-x0)x(x2-x0)/|.|).  The mesh must be conforming, with no point contacts (footnote in
 *     Section 4.3) and no two triangles at an edge lying in the same half-plane.
 *   - Degrees of freedom: one per generalized vertex x_{i,j} with j < q_i (eq.
 *     defCurlyHtildeGamma), in canonical order (vertex index, then sector label); sector labels
 *     at a vertex are ordered by their smallest member (triangle index, side + before side -),
 *     the last sector is the reference one of eq. defYij.  Side + of T is where n_T points.
 *   - Oriented triangles carry the outward normal of the sector they bound:
 *     n_(T,+) = -n_T, n_(T,-) = +n_T.
 *   - All host arrays are caller-owned and only read (inputs, copied during the call) or written
 *     (outputs, caller-allocated) during the call.  Handles are freed with *_destroy.  A problem
 *     must outlive its preconditioners.  All calls return 0 (BEM_OK) or a negative error code;
 *     bem_last_error() gives the thread-local message of the last failing call.
 *   - Every step of the compute path runs in HIP kernels on the context's device; there is no
 *     CPU fallback.
 */
#ifndef BEM_H_
#define BEM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BEM_OK = 0,
    BEM_PENDING = 1,                 /* bem_serve_poll: request still running */
    BEM_E_INVALID_ARG = -1,
    BEM_E_MESH_NONCONFORMING = -2,   /* repeated vertices/triangles, coincident pages at an edge */
    BEM_E_DEGENERATE = -3,           /* zero-area triangle */
    BEM_E_POINT_CONTACT = -4,        /* triangles at a vertex not connected through edges */
    BEM_E_NOT_SPD = -5,              /* Cholesky pivot <= 0 in a preconditioner block */
    BEM_E_BREAKDOWN = -6,            /* p.Wp <= 0 or NaN in (P)CG */
    BEM_E_NOT_CONVERGED = -7,        /* max_iter reached; outputs are still written */
    BEM_E_ADMISSION = -8,            /* request larger than the HBM budget */
    BEM_E_OOM = -9,
    BEM_E_DEVICE = -10,              /* HIP runtime error */
    BEM_E_UNSUPPORTED = -11
};

typedef struct bem_ctx bem_ctx;
typedef struct bem_problem bem_problem;
typedef struct bem_precond bem_precond;
typedef struct bem_server bem_server;

typedef enum { BEM_FP64 = 0, BEM_FP32_REFINE = 1 } bem_precision;

typedef struct {
    bem_precision precision; /* BEM_FP32_REFINE also keeps an FP32 copy of W for inner solves */
    int near_order;          /* Gauss-Legendre points per axis in the Duffy rules (default 10) */
    int keep_pair_matrix;    /* 1: keep I(T,T') on the device for bem_problem_pair_integrals */
    int64_t pair_panel_rows; /* 0: automatic; > 0: assemble through panels of the pair matrix with at
                              * most this many triangle rows (the automatic choice uses panels only
                              * when the whole N_T x N_T pair matrix does not fit next to W) */
    int32_t keep_order;      /* 0 (default): the problem numbers vertices and triangles internally in
                              * Morton order of their positions (compact blocks of consecutive dofs
                              * for the contraction); 1: it keeps the caller's numbering.  Either way
                              * every call takes and returns dof-, vertex- and triangle-indexed data
                              * in the caller's numbering and canonical dof order. */
} bem_assemble_opts;

typedef struct {
    int64_t n_dofs, n_tri, n_vert, n_near_pairs;
    int64_t bytes_device;    /* device memory held by the problem */
    int64_t q_hist[16];      /* number of vertices with q sectors (q >= 15 in the last bin) */
    double t_assemble_s;     /* wall time of bem_assemble: it returns once the device has consumed the
                                inputs; the contraction into W (panel-by-panel assembly: the panels)
                                may still run (later calls on the problem queue behind it, and the
                                copy calls wait for it) */
    double t_far_s, t_near_s, t_contract_s; /* device time of the three assembly phases (NaN while that
                                                device work still runs) */
    double t_host_s;         /* host time of the mesh analysis and near-pair list */
    int64_t n_pair_panels;   /* panels the pair matrix was built in (0: in one piece) */
    int64_t dim;             /* 3: triangle mesh (n_tri triangles); 2: segment mesh (n_tri segments) */
    int64_t panels_replanned; /* panels are laid out before the sector analysis, from the sector count
                               * q = T_v - E_v + 2 that the numbers of triangles and edges at each
                               * vertex give (Euler's formula for the graph they cut on a small
                               * sphere about it); 1: the analysis numbered the dofs otherwise and
                               * the panels were planned again (0 for every mesh it accepts) */
} bem_problem_info;

typedef struct {
    int use_coarse;          /* 1: add the coarse-space correction (default 1) */
    int factor_fp32;         /* 1: store block inverses in FP32 (mixed-precision inner solves) */
    int wirebasket;          /* 0: exact Galerkin block of the wire basket (default); 1: its
                              * diagonal, the pointwise product of Remark "Approximate solvers"
                              * (Section 2), applied as R_W^T diag(W_WW)^{-1} R_W */
    double diag_shift;       /* sigma added to the diagonal of every face, wire-basket and coarse
                              * block before it is factorised (W_XX + sigma I; default 0).  A
                              * positive shift regularises the local solvers; a shift below minus
                              * the smallest eigenvalue of a block makes it indefinite, and the
                              * set-up then fails with BEM_E_NOT_SPD. */
} bem_precond_opts;

typedef struct {
    double tol;              /* stop when ||L - W x||_2 <= tol ||L||_2 per column (1e-10) */
    int max_iter;            /* total (P)CG iterations per column (default 2000) */
    int use_precond;         /* 0: plain CG even if a preconditioner is passed */
    bem_precision precision; /* BEM_FP32_REFINE: FP32 matrix/factors inside FP64 refinement */
    double refresh_factor;   /* mixed precision: replace the recurrence residual by the FP64 residual
                              * b - W x each time it has fallen by this factor; 0 (or outside (0, 1)):
                              * the default 2.5e-4, about the square root of FP32's unit roundoff */
    int check_every;         /* iterations between host convergence checks (default 4) */
    int use_graph;           /* 1: replay one captured iteration with hipGraphLaunch */
    const double* x0;        /* NULL: x0 = 0; else host memory holding k x N start vectors
                              * (column-major, column c at x0 + c N, canonical dof order); the
                              * first residual is then L - W x0 with the FP64 matrix */
} bem_solve_opts;

typedef struct {
    int iters;               /* (P)CG iterations (products with W) of this column */
    int outer_iters;         /* FP64 residual recomputations (mixed precision) */
    int status;              /* BEM_OK / BEM_E_NOT_CONVERGED / BEM_E_BREAKDOWN */
    int graph;               /* 1: iterations replayed from captured graphs; 0: launched directly
                              * (use_graph = 0, or a capture the HIP runtime broke off because of a
                              * call elsewhere in the process; same kernels, same results) */
    double relres;           /* final ||L - W x|| / ||L|| with the FP64 matrix */
    double est_cond;         /* Lanczos estimate of kappa(M W) from the (P)CG coefficients */
    double t_total_s;        /* wall time of the whole call; served requests: submit to completion */
    double t_start_s;        /* served requests: submit to the start of the request's columns in a
                              * block PCG (queueing, plus assembly and set-up of a geometry that was
                              * not resident); 0 for bem_pcg_solve */
} bem_solve_info;

/* ---- context ------------------------------------------------------------------------------ */
/* Binds the calling library instance to HIP device `hip_device`.  hbm_budget_bytes limits the
 * device memory the serving loop may hold (0 = 90% of free memory). */
int bem_ctx_create(int hip_device, size_t hbm_budget_bytes, bem_ctx** out);
/* Launch parameters of the kernels, chosen per size class by the autotuner of this project
 * (paper_2310_09204_amd/tune.py, measured on the device) and handed over with bem_ctx_set_tuning.
 * None of them changes a result beyond rounding: the separation factor s decides which column
 * groups the far-field kernel evaluates in its centred form, whose rounding of |x - y|^2 grows like
 * ((s + 1) / (s - 1))^2 ulp, so s >= 1.1 keeps it below 1e-13 relative.  A zero field takes the
 * default. */
typedef struct {
    int64_t max_triangles;     /* the entry covers meshes of up to this many triangles (the last
                                  entry covers every larger mesh as well) */
    double far_separation;     /* centred far-field form when column groups are this many times the sum
                                  of the two Gauss-point radii apart, in [1.1, 3]; default 1.2 */
    double panel_fraction;     /* share of the free device memory for the pair-matrix panels of
                                  panel-by-panel assembly, in [0.2, 0.8]; default 0.6 */
    int32_t symv_blocks_fp64;  /* super-block edge (64-row blocks) of the symmetric product with the
                                  FP64 matrix: 2, 4 or 8; default 4 */
    int32_t symv_blocks_fp32;  /* the same for the FP32 copy: 4, 8 or 16; default 8 */
    int32_t check_every;       /* PCG iterations between host checks when bem_solve_opts leaves
                                  check_every at 0; default 4 */
    int32_t reserved;
} bem_tuning;
/* Copies n entries (sorted by max_triangles, n <= 16; n = 0 restores the defaults).  Problems
 * assembled afterwards take the first entry whose max_triangles holds their mesh.  Errors:
 * BEM_E_INVALID_ARG for a value outside the ranges above. */
int bem_ctx_set_tuning(bem_ctx* ctx, const bem_tuning* entries, int32_t n);
/* The entry (defaults filled in) that a problem was assembled with. */
int bem_problem_tuning(const bem_problem* p, bem_tuning* out);
void bem_ctx_destroy(bem_ctx* ctx);
/* Waits for all device work of the context's device (hipDeviceSynchronize). */
int bem_ctx_synchronize(bem_ctx* ctx);
/* Device buffers the library frees are kept per device for reuse (a stream-ordered cache, shared
 * by all contexts of the device).  This returns them to the HIP runtime; it waits for the
 * buffers' last users and serialises with graph captures of concurrent solves.  Only memory no
 * live problem or preconditioner holds is released.  Returns BEM_OK or BEM_E_DEVICE. */
int bem_ctx_release_cached(bem_ctx* ctx);

/* ---- host-side mesh analysis (no device work) --------------------------------------------- */
/* Sectors and dofs of Section 4.2 for a mesh: returns the number of dofs in *n_dofs and, if the
 * arrays are non-NULL, the dof table (dof_vertex[N], dof_sector[N]) and the per-vertex sector
 * counts q[nv].  Validation errors as for bem_assemble. */
int bem_mesh_analyze(const double* vertices, int64_t nv, const int32_t* triangles, int64_t nt,
                     int64_t* n_dofs, int32_t* dof_vertex, int32_t* dof_sector, int32_t* q);

/* ---- assembly (Section 4.3, eq. eval_a_phiij with Cor. corW) ------------------------------- */
/* Builds the dense Galerkin matrix on the device:
 *   W_{d,d'} = sum_{T,T'} I(T,T') J_{T,d} . J_{T',d'},  I(T,T') = 1/(4 pi) int_T int_T' |x-y|^{-1},
 *   J_{T,d} = sum_a c_{T,a,d} (x_{a+1} - x_{a+2}) / (2|T|)   (surface curl of the trace jump).
 * I uses a 7-point degree-5 rule on each triangle of pairs with no common vertex and
 * Duffy-regularised Gauss-Legendre rules (near_order points per axis) on pairs with a common
 * vertex, edge, or triangle.  W is stored FP64 row-major; with BEM_FP32_REFINE also as FP32.
 * The call returns once the device has read the inputs; the last kernel (the contraction into W)
 * may still be running then.  Every later call on the problem is ordered after it.
 * Errors: BEM_E_INVALID_ARG, BEM_E_DEGENERATE, BEM_E_MESH_NONCONFORMING, BEM_E_POINT_CONTACT,
 * BEM_E_OOM, BEM_E_DEVICE (a fault of the unfinished contraction surfaces in a later call). */
int bem_assemble(bem_ctx* ctx, const double* vertices, int64_t nv, const int32_t* triangles,
                 int64_t nt, const bem_assemble_opts* opts, bem_problem** out);
/* The same assembly with the mesh also resident on the device: vertices / triangles (host) feed
 * the host-side analysis (sectors, dofs, near pairs, plans), d_vertices / d_triangles (device
 * memory of the context's device, same layout and values) feed the kernels, so no mesh upload
 * happens in the call.  The device arrays are read on the library's streams: the caller's writes
 * to them must be complete before the call (e.g. a device synchronisation); they may be freed
 * after it returns.  Errors as for bem_assemble; values identical to bem_assemble's. */
int bem_assemble_dev(bem_ctx* ctx, const double* vertices, const double* d_vertices, int64_t nv,
                     const int32_t* triangles, const int32_t* d_triangles, int64_t nt,
                     const bem_assemble_opts* opts, bem_problem** out);
void bem_problem_destroy(bem_problem* p);
int bem_problem_get_info(const bem_problem* p, bem_problem_info* info);
/* dof table in canonical order: vertex index and sector label of each dof */
int bem_problem_dofs(const bem_problem* p, int32_t* dof_vertex, int32_t* dof_sector);
/* rows row0 .. row0+nrows-1 of W (FP64) into out[nrows][N] */
int bem_problem_copy_matrix(const bem_problem* p, int64_t row0, int64_t nrows, double* out);
/* selected rows of W into out[nrows][N] */
int bem_problem_copy_rows(const bem_problem* p, const int64_t* rows, int64_t nrows, double* out);
/* I(T,T') for npairs index pairs (int32[npairs][2]); needs keep_pair_matrix = 1 */
int bem_problem_pair_integrals(const bem_problem* p, const int32_t* pairs, int64_t npairs,
                               double* out);
/* right-hand side L (eq. defRhs, constant g): L_d = -sum_T (g.n_T) c_{T,a,d} |T|/3, k columns,
 * out[k][N] (column-major, one column per g) */
int bem_rhs(const bem_problem* p, const double* g, int32_t k, double* out);
/* y = W x for k column vectors x[k][N] -> y[k][N] (FP64 matrix, or FP32 matrix if fp32 = 1).
 * Columns go in groups of 16; each group reads only the upper block triangle of the symmetric W
 * (each 64 x 64 block applied to both sides); a matrix of a single 64-row block is streamed whole.
 * Sums run in a fixed order: equal inputs give bit-identical outputs. */
int bem_matvec(const bem_problem* p, const double* x, int32_t k, int fp32, double* y);
/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): y = W x as bem_matvec, with d_x and d_y device pointers
 * ([k][N] each, column-major, leading dimension N, caller-owned), that calls no hipMalloc,
 * hipFree or other allocating routine.  The transposed right-hand sides and the partial sums of
 * the product live in one static device array of 128 MiB per device (held from the library's
 * first use on that device until the process ends; its address is looked up in bem_ctx_create).
 * A product needs 16 N s + (N/64) (ceil(N/256 or N/512) + 1) 1024 s bytes of it (s = 8, or 4
 * with fp32 = 1, N rounded up to 64; super-blocks of 4 FP64 or 8 FP32 blocks; with a renumbered
 * problem also x and y in its internal dof order): N up to 15,872 (FP64) or 31,232 (FP32) at
 * k = 16, 16,064 / 32,128 at k = 1; larger products get BEM_E_INVALID_ARG and must use bem_matvec.  Runs on the problem's stream and returns when y is written.  Every call
 * on one device shares the array, which keeps the last call's contents: calls that overlap on
 * one device race (calls on one problem are serialised).  Errors: BEM_E_INVALID_ARG (NULL, k < 1,
 * fp32 without an FP32 matrix, scratch too small), BEM_E_DEVICE. */
int bem_matvec_noalloc(const bem_problem* p, const double* d_x, int32_t k, int fp32, double* d_y);
/* Measurement: `reps` back-to-back products y = W x with k device-resident columns (FP64 matrix,
 * or the FP32 copy if fp32 = 1), timed with HIP events on the problem's stream; writes the mean
 * seconds per product.  The upper block triangle of W is read plus the block-row partials of the
 * symmetric product, for any k (a matrix of one 64-row block: N^2 x 8 or 4 bytes). */
int bem_problem_bench_matvec(const bem_problem* p, int fp32, int32_t k, int reps, double* seconds);
/* label-free view of phi[N]: jump[t][a] = sum_d c_{T,a,d} phi_d, the jump of the represented
 * function across triangle t at corner a (jump_out[nt][3]); for a segment mesh across segment s
 * at its end a (jump_out[ns][2]) */
int bem_jump_values(const bem_problem* p, const double* phi, double* jump_out);

/* ---- two-dimensional variant (Section 2, Experiments 1 and 2) ---------------------------- */
/* Segment multiscreens in the plane: vertices[nv][2], segments[ns][2]; the order of a segment's
 * ends fixes its tangent tau_s and normal n_s = (-tau_y, tau_x).  Sectors at a vertex are the
 * angular regions between its segments (a segment end no other segment meets has q = 1 and no
 * dof); dofs, the jump basis and the coefficients c_{s,a,d} follow Section 4.2 with segments for
 * triangles.  W_{d,d'} = sum_{s,s'} D_{s,d} D_{s',d'} K(s,s') with D_{s,d} = (c_{s,1,d} -
 * c_{s,0,d}) / |s| (derivative of the jump along s) and K(s,s') = -1/(2 pi) int_s int_s' log|x-y|:
 * 8-point Gauss-Legendre on both segments of a disjoint pair, a closed form for a segment with
 * itself, and for segments with a common end the split of the parameter square along its
 * diagonal with the singular factor integrated exactly.  The problem works with bem_pcg_solve
 * (g[k][3] with g_z ignored: L_d = -sum_s (g . n_s) |s| / 2 (c_{s,0,d} + c_{s,1,d})),
 * bem_pcg_solve_rhs, bem_rhs, bem_matvec, bem_problem_copy_matrix, bem_problem_rows,
 * bem_jump_values, bem_problem_bench_matvec, bem_double_layer and bem_precond_setup_2d;
 * bem_precond_setup rejects it.  opts: precision as for bem_assemble (near_order is not used).
 * Errors: BEM_E_INVALID_ARG (NULL, index out of range, non-finite coordinate), BEM_E_DEGENERATE
 * (zero length), BEM_E_MESH_NONCONFORMING (repeated or overlapping segments), BEM_E_OOM,
 * BEM_E_DEVICE.  K takes ns^2 x 8 bytes of device memory during the call. */
/* Host-only analysis of a segment mesh: *n_dofs, and if non-NULL the dof table (dof_vertex[N],
 * dof_sector[N]), the per-vertex sector counts q[nv] and the jump coefficients as a dense
 * array c[ns][2][N] (c_{s,a,d}; only for small meshes).  Validation errors as bem_assemble_2d. */
int bem_mesh_analyze_2d(const double* vertices, int64_t nv, const int32_t* segments, int64_t ns, int64_t* n_dofs,
                        int32_t* dof_vertex, int32_t* dof_sector, int32_t* q, double* c);
int bem_assemble_2d(bem_ctx* ctx, const double* vertices, int64_t nv, const int32_t* segments, int64_t ns,
                    const bem_assemble_opts* opts, bem_problem** out);

/* The substructuring preconditioner of bem_precond_setup for a segment mesh (eq. jumpSplit in two
 * dimensions): face dofs of patch P are the dofs at vertices whose segments all have
 * patch_of_segment == P and with q = 2, the rest is the wire basket, and the coarse space is the
 * jump space of the nested coarse segment mesh (coarse_vertices[ncv][2], coarse_segments[ncs][2]),
 * coarse_of_segment[s] being the coarse segment that contains fine segment s.  The coarse jump
 * basis is written in the fine basis from the coarse hat functions, minus the mean over the
 * sectors at each fine vertex.  Options, errors and the result as for bem_precond_setup; the
 * problem must come from bem_assemble_2d. */
int bem_precond_setup_2d(bem_problem* p, const int32_t* patch_of_segment, const double* coarse_vertices, int64_t ncv,
                         const int32_t* coarse_segments, int64_t ncs, const int32_t* coarse_of_segment,
                         const bem_precond_opts* opts, bem_precond** out);

/* ---- double-layer potential (Lemma repDL, eq. formulaDL) --------------------------------- */
/* U_c(x_i) = sum_T int_T n_T . (x_i - y) / (4 pi |x_i - y|^3) [u_c]_T(y) dsigma(y) for the solution
 * columns phi[c] (c < k) of this problem, where [u_c]_T is the jump across T of sum_d phi[c][d]
 * psi_d (the per-corner values of bem_jump_values, linear on T).  The sides' normals follow the
 * orientation of bem_pcg_solve (side + has the outward normal -n_T), so U jumps by [u] across the
 * screen.  The integral is the 7-point rule on every triangle: accurate for targets at least a few
 * mesh sizes from the screen, with no refinement closer in.  phi: host [k][N]; targets: host
 * [m][3]; u_out: host [k][m].  Per-triangle data are built on the first call and kept with the
 * problem.  For a segment mesh (bem_assemble_2d): U_c(x) = sum_s int_s n_s . (x - y) /
 * (2 pi |x - y|^2) [u_c]_s(y) dy with 8-point Gauss-Legendre on every segment, targets[m][3] with
 * the third coordinate ignored.  Returns BEM_OK, or BEM_E_INVALID_ARG (NULL pointer, k < 1, m < 0,
 * non-finite target), BEM_E_OOM, BEM_E_DEVICE. */
int bem_double_layer(bem_problem* p, const double* phi, int32_t k, const double* targets, int64_t m,
                     double* u_out);

/* ---- preconditioner (eq. jumpSplit; Remark on PCG iterations) ------------------------------ */
/* Two-level additive Schwarz operator
 *   M r = sum_F R_F^T W_FF^{-1} R_F r + R_W^T W_WW^{-1} R_W r + R_H^T (R_H W R_H^T)^{-1} R_H r.
 * Face dofs of patch P: dofs at vertices whose triangles all have patch_of_triangle == P and with
 * q = 2; all other dofs form the wire basket.  The coarse space is the jump space of the nested
 * coarse mesh (coarse_vertices, coarse_triangles); coarse_of_triangle[t] is the coarse triangle
 * containing fine triangle t.  Pass ncv = 0 for no coarse space.  Patch ids < 0 put their
 * vertices in the wire basket.  Errors: BEM_E_INVALID_ARG, BEM_E_NOT_SPD, mesh errors of the
 * coarse mesh, BEM_E_OOM, BEM_E_DEVICE. */
int bem_precond_setup(bem_problem* p, const int32_t* patch_of_triangle,
                      const double* coarse_vertices, int64_t ncv, const int32_t* coarse_triangles,
                      int64_t nct, const int32_t* coarse_of_triangle, const bem_precond_opts* opts,
                      bem_precond** out);
void bem_precond_destroy(bem_precond* m);
/* sizes: number of face blocks, wire-basket size, coarse dofs, largest face block */
int bem_precond_sizes(const bem_precond* m, int64_t* n_faces, int64_t* n_wb, int64_t* n_coarse,
                      int64_t* max_face);
/* z = M r for k columns r[k][N] -> z[k][N] (FP64 factors) */
int bem_precond_apply(const bem_precond* m, const double* r, int32_t k, double* z);

/* ---- solve (Remark "Bound on the number of Preconditioned Conjugate Gradient iterations") -- */
/* Solves W Phi = L for k constant Neumann vectors g[k][3] by (P)CG from x0 = 0 (or opts->x0),
 * preconditioned by M if m != NULL and opts->use_precond.  FP64 mode: W, vectors and factors in
 * FP64.  BEM_FP32_REFINE: PCG with products by the FP32 matrix and FP32 block inverses (FP64
 * vectors, dots, updates and coarse solve) and reliable updates: the recurrence residual is replaced
 * by the true residual L - W x with the FP64 matrix each time it has fallen by refresh_factor, and
 * a column counts as converged only when a true residual satisfies ||r|| <= tol ||L||
 * (info.outer_iters = number of replacements).  phi_out[k][N] column-major.  Returns BEM_OK,
 * BEM_E_NOT_CONVERGED or BEM_E_BREAKDOWN (outputs written in all three cases). */
int bem_pcg_solve(bem_problem* p, const bem_precond* m, const double* g, int32_t k,
                  const bem_solve_opts* opts, double* phi_out, bem_solve_info* info);
/* Same for explicit right-hand sides rhs[k][N]. */
int bem_pcg_solve_rhs(bem_problem* p, const bem_precond* m, const double* rhs, int32_t k,
                      const bem_solve_opts* opts, double* phi_out, bem_solve_info* info);
/* bem_pcg_solve with the solution left on the device: d_phi_out is device memory of the
 * context's device holding k x N doubles (column c at d_phi_out + c N), written when the call
 * returns (the problem's stream is synchronised).  info, g and the errors as for bem_pcg_solve. */
int bem_pcg_solve_dev(bem_problem* p, const bem_precond* m, const double* g, int32_t k,
                      const bem_solve_opts* opts, double* d_phi_out, bem_solve_info* info);

/* ---- serving loop ------------------------------------------------------------------------- */
/* A background host thread takes solve requests on arbitrary multiscreens, keeps assembled
 * problems and preconditioners resident (keyed by a hash of mesh + partition + coarse mesh),
 * admits a request when its device footprint (N^2 x bytes per entry + blocks) fits the context's
 * budget next to everything resident, and runs up to max_inflight geometries at once on their own
 * HIP streams.  Continuous batching: a geometry runs as one block PCG on column slots (16, or the
 * columns of the requests queued when it starts); requests on the same geometry and precision
 * that arrive while it assembles or solves join it and start in the slots that finished columns
 * free up, each column with its own tolerance; a request completes when its own columns have
 * stopped.  Its info[c].relres is the residual the iteration tracked (the true residual for
 * BEM_FP32_REFINE, the recurrence residual for BEM_FP64). */
int bem_server_create(bem_ctx* ctx, int max_inflight, bem_server** out);
void bem_server_destroy(bem_server* s);
typedef struct {
    const double* vertices; int64_t nv;
    const int32_t* triangles; int64_t nt;
    const int32_t* patch_of_triangle;
    const double* coarse_vertices; int64_t ncv;
    const int32_t* coarse_triangles; int64_t nct;
    const int32_t* coarse_of_triangle;
    const double* g; int32_t k;
    bem_precision precision;
    double tol;
} bem_request;
/* Copies the request's arrays and queues it; *ticket identifies it.  BEM_E_ADMISSION if it can
 * never fit the budget. */
int bem_serve_submit(bem_server* s, const bem_request* req, uint64_t* ticket);
/* Waits up to timeout_us (-1 = forever) for the request; BEM_PENDING if not finished.  On
 * completion writes phi_out[k][N] and info[k] (if non-NULL) and releases the ticket. */
int bem_serve_poll(bem_server* s, uint64_t ticket, int64_t timeout_us, double* phi_out,
                   bem_solve_info* info);
/* The number of dofs of a submitted request (so the caller can size phi_out). */
int bem_serve_ndofs(bem_server* s, uint64_t ticket, int64_t* n_dofs);
typedef struct {
    int64_t submitted, completed, rejected, merged_batches, cache_hits, cache_misses;
    int64_t resident_bytes, peak_resident_bytes, evictions;
    int64_t admitted_running;   /* requests that joined a block PCG already running on their geometry */
} bem_server_stats;
int bem_server_get_stats(bem_server* s, bem_server_stats* st);

const char* bem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BEM_H_ */
