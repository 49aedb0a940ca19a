/*
 * ebamg.h -- C ABI of the MI355X (gfx950) embedded-boundary AMG-PCG library.
 *
 * The library solves the symmetric positive definite system A u = b that the
 * line-by-line embedded-boundary discretisation of -Laplace produces on a
 * uniform Cartesian node grid (Peng, Appelo, Liu, "Universal AMG accelerated
 * embedded boundary method without small cell stiffness"; Algorithm 2):
 *
 *   step 1  classify nodes (mask, boundary points, computational points);
 *   steps 2-3  central differences with the Dirichlet condition imposed by
 *           interpolating to interior boundary points along grid lines, which
 *           changes only the diagonal and the right-hand side;
 *   step 4  conjugate gradients preconditioned by algebraic multigrid.
 *
 * A = (1/h^2) (diag(a) - adjacency of computational points) + sigma I, where
 * the dimensionless diagonal is a_k = (number of computational neighbours) +
 * sum over boundary-point sides of 1/q, q*h being the distance from the
 * computational point to the boundary crossing on that grid line (Sec. 2.1.1).
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - Node fields are dense (n[0]+1) x (n[1]+1) [x (n[2]+1)] arrays, x fastest
 *     (flat index i + nx*(j + ny*k)), no padding.
 *   - The caller owns every array it passes; the library owns only the
 *     amg_handle_t and the memory it allocated for it.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on that stream unless stated otherwise.
 *   - Return 0 on success or a negative EB_E* code; eb_last_error() returns a
 *     thread-local message for the last failure.  No exception or abort crosses
 *     the ABI.  Outputs are unspecified after an error unless stated.
 *   - Inside the domain means psi < 0 strictly; psi == 0 is outside.
 *   - Everything is FP64.
 */
#ifndef EBAMG_H
#define EBAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBAMG_ABI_VERSION 1

enum {
    EB_OK = 0,
    EB_EINVAL = -1,    /* bad argument (null pointer, dim, sizes, params)        */
    EB_EDOMAIN = -2,   /* an outermost-layer node is inside (psi < 0)             */
    EB_ENOSPC = -3,    /* an output capacity is too small (required size is
                          still reported where the call says so)                 */
    EB_ENOTSPD = -4,   /* non-positive pivot / curvature: operator not SPD       */
    EB_ENAN = -5,      /* NaN or Inf met in the solve                             */
    EB_ENOCONV = -6,   /* maxit reached before the tolerance                      */
    EB_EHIP = -7,      /* a HIP runtime call failed                               */
    EB_ENOTIMPL = -8,  /* feature not available                                   */
    EB_EGEOM = -9      /* an RBF row's interpolation points are collinear         */
};

/* Boundary-condition strategy of the assembly (Sec. 2.3, Algorithm 2 step 3). */
enum {
    EB_BC_LINE = 0,    /* line-by-line on every boundary-point side; where the node
                          two steps out is inside, the grid line is followed to
                          the first outside node (extended line-by-line)        */
    EB_BC_MIXED = 1,   /* "mixed": line-by-line where the node two steps out is
                          outside, RBF interpolation otherwise (2-D only)        */
    EB_BC_RBF = 2      /* "RBF-based": RBF interpolation on every side (2-D only) */
};

/* Node grid: node (i,j,k) sits at x0 + (i,j,k)*h, i = 0..n[0] etc. (host struct) */
typedef struct {
    int32_t dim;       /* 2 or 3                                                  */
    int32_t n[3];      /* cells per axis; n[2] ignored when dim == 2              */
    double x0[3];      /* coordinates of node 0; x0[2] ignored when dim == 2      */
    double h;          /* spacing, > 0                                            */
} eb_grid_t;

/* One boundary point used by a boundary-point side of a computational point.
 * A line-by-line side (Sec. 2.1.1) has one record: the crossing of its grid
 * line, weight c = 1/q.  An RBF side (Sec. 2.2) has two: the boundary points
 * x_Gamma1, x_Gamma2 of Algorithm 1 with the RBF interpolant's weights.  The
 * side adds the sum of its records' c to the diagonal, and every record adds
 * u(xg) c / h^2 to the right-hand side.  Records are sorted by (node, dir,
 * point).                                                                      */
typedef struct {
    int64_t node;      /* flat node index of the computational point            */
    int32_t dir;       /* side: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z               */
    int32_t steps;     /* line-by-line: j >= 2, node + j*side is the first outside
                          node; RBF: -1 for x_Gamma1, -2 for x_Gamma2            */
    double q;          /* line-by-line: crossing distance / h, in (1, j]; RBF: 0 */
    double c;          /* line-by-line: 1/q (weight g_Gamma of the crossing);
                          RBF: the interpolant's weight of this boundary point  */
    double xg[3];      /* boundary point coordinates (xg[2] = 0 in 2-D)          */
} eb_cut_t;            /* 56 bytes                                               */

/* Optional device allocator for a handle (see amg_params_t): alloc returns
 * `bytes` of device memory usable in stream order on `stream` (NULL on
 * failure); free releases a block in stream order on `stream`.             */
typedef void* (*eb_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*eb_free_fn)(void* ptr, void* stream, void* ctx);

typedef struct {
    int32_t coarse_max;      /* solve densely once n <= coarse_max (default 256)  */
    int32_t max_levels;      /* hierarchy depth limit (default 16)                */
    double min_reduction;    /* stop coarsening if n_next > min_reduction * n (0.6) */
    int32_t dense_limit;     /* refuse a dense coarsest level above this (default
                                and upper bound 1200: the factorisation keeps a
                                16-column panel of the level in LDS)           */
    int32_t reserved;
    eb_alloc_fn alloc;       /* both set: every device block the library takes
                                during amg_setup and during later calls on the
                                handle (solves, V-cycle and smoother calls,
                                amg_free) comes from alloc and goes back through
                                free, with the stream of the call (e.g. a
                                framework's caching allocator).  Both NULL: the
                                library's own caching allocator.  One of them
                                NULL: EB_EINVAL.                               */
    eb_free_fn free;
    void* alloc_ctx;         /* passed to alloc and free                         */
} amg_params_t;

typedef struct {
    double tol;              /* stop when ||r||_2 <= tol * ||b||_2                */
    int32_t maxit;           /* iteration limit (default 1000)                    */
    int32_t x0_given;        /* 1: x holds the initial guess on entry; 0: x0 = 0  */
    int32_t check_every;     /* iterations queued between convergence polls (8)   */
    int32_t precision;       /* V-cycle precision: EB_PREC_FP64 (0, default),
                                EB_PREC_FP32 (1: single-precision V-cycle; the
                                outer CG, its dot products, the true-residual
                                check with restart and the coarsest dense
                                solve stay FP64) or EB_PREC_BF16 (2: that
                                V-cycle with the BF16 fine smoother below).
                                Hierarchies of one level always run FP64.      */
} pcg_params_t;

enum { EB_PREC_FP64 = 0, EB_PREC_FP32 = 1, EB_PREC_BF16 = 2 };
/* EB_PREC_BF16: the single-precision V-cycle of EB_PREC_FP32 whose fine-level
 * smoother runs on BF16 operands: it scales by a BF16 copy of 1/diag and
 * stores the preconditioned residual z in BF16 (round to nearest even);
 * its arithmetic is FP32 and the outer CG stays FP64.  Not with per-point
 * smoother weights (EB_ENOTIMPL) or in batched solves (EB_EINVAL).          */

typedef struct {
    int32_t iterations;      /* products with A inside CG                         */
    int32_t status;          /* EB_OK, EB_ENOCONV, EB_ENOTSPD or EB_ENAN          */
    int32_t restarts;        /* restarts after true-residual drift (0 or 1)       */
    int32_t levels;          /* hierarchy depth used                              */
    double rel_res_recursive;/* ||r_k|| / ||b|| of the recursive residual         */
    double rel_res_true;     /* ||b - A x|| / ||b||, recomputed at exit           */
    double solve_ms;         /* device time of the solve (HIP events)             */
    double reserved;
} pcg_result_t;

typedef struct amg_handle amg_handle_t;

/* Per-level description returned by amg_level_info (host struct).  The device
 * pointers stay owned by the handle and are valid until amg_free.            */
typedef struct {
    int64_t n;               /* unknowns on this level                           */
    int64_t nnz_a, nnz_p, nnz_r;
    double rho;              /* Gershgorin bound of D^-1 A (0 on the coarsest)   */
    double omega;            /* 4 / (3 rho)                                      */
    int32_t is_coarsest;
    int32_t max_comp;        /* most aggregates sharing one box on this level    */
    int32_t ext[3];          /* coordinate extents of this level                 */
    int32_t nnz_ap;          /* entries of A P, stored with its transpose R A for the
                                V-cycle (0 on the coarsest and on level 0)         */
    const int32_t* a_rowptr; const int32_t* a_col; const double* a_val;
    const int32_t* p_rowptr; const int32_t* p_col; const double* p_val;
    const int32_t* r_rowptr; const int32_t* r_col; const double* r_val;
    const int32_t* agg;      /* aggregate (coarse unknown) of each unknown       */
    const int32_t* coords;   /* n x 3 integer coordinates                         */
    const double* dense_inv; /* coarsest only: n x n inverse, row-major          */
} amg_level_info_t;

/* Step 1 and the diagonal of steps 2-3 (Sec. 2 definitions; Sec. 2.1.1
 * interpolant; the crossing is the root of psi on the grid line, Sec. 2.1.1,
 * located here by linear interpolation of psi between the last inside and the
 * first outside node, the second-order distance approximation of Sec. 3.3).
 *   psi   [in]  node field, level set, negative inside.
 *   kind  [out] node field int8: 0 outside, 1 boundary point, 2 computational.
 *   a     [out] node field: a_k at computational points, 0 elsewhere.
 *   cuts  [out] up to cuts_cap records, sorted by (node, dir); may be NULL
 *               when cuts_cap == 0.
 *   n_unknowns, n_cuts [host out] totals, always written on EB_OK and
 *               EB_ENOSPC (cuts_cap < *n_cuts: records beyond cuts_cap are
 *               not written).
 * Synchronises `stream` to return the counts.  EB_EDOMAIN if an outermost
 * node is inside.  When the node two steps beyond a computational point is
 * itself inside, the grid line is followed to the first outside node and the
 * same two-point interpolation is used (q may exceed 2).                       */
int eb_assemble_diag(const eb_grid_t* g, const double* psi, int8_t* kind, double* a,
                     eb_cut_t* cuts, int64_t cuts_cap, int64_t* n_unknowns,
                     int64_t* n_cuts, void* stream);

/* eb_assemble_diag with a choice of boundary treatment (Sec. 2.3; Algorithm 2
 * step 3): mode EB_BC_LINE is eb_assemble_diag; EB_BC_MIXED and EB_BC_RBF
 * impose the condition on some or all boundary-point sides by the RBF
 * interpolant of Sec. 2.2 (Eq. (rbf), (rbf_ubp), phi(r) = r^3 with linear
 * polynomials, Sec. 3), whose two boundary points follow Algorithm 1:
 * x_Gamma1 closest to the BP, x_Gamma2 closest to the computational point,
 * or, when the two are within epsilon h (epsilon = 0.025), the first point of
 * Gamma on the ray from the BP turned pi/4 counterclockwise from x_Gamma1.
 * Gamma is the zero set of the piecewise-linear interpolant of psi on the
 * triangles that split every cell along its (i,j)-(i+1,j+1) diagonal; the
 * closest points are searched in the 6h x 6h window of cells around the
 * computational point, which holds them (the BP is within h of Gamma).
 * With three points and linear polynomials the interpolant is the linear
 * one through them, so the weights are barycentric coordinates (evaluated in
 * units of h relative to the computational point).  Such a side writes two
 * records (steps -1, -2).  Only the diagonal and the right-hand side change,
 * so the operator stays symmetric; definiteness is not guaranteed (check it
 * with eb_check_spd).
 * EB_EINVAL for an unknown mode, EB_ENOTIMPL for RBF modes in 3-D, EB_EGEOM
 * when a side's three interpolation points are collinear; otherwise as
 * eb_assemble_diag.                                                          */
int eb_assemble_diag_mode(const eb_grid_t* g, const double* psi, int32_t mode, int8_t* kind, double* a,
                          eb_cut_t* cuts, int64_t cuts_cap, int64_t* n_unknowns,
                          int64_t* n_cuts, void* stream);

/* eb_assemble_diag_mode for a variable conductivity beta (Eq. (1), with the
 * face values beta_{i+-1/2} of Eq. (central_difference)).  beta [in]: dim
 * node fields back to back (device), field `axis` holding beta at the
 * midpoint of the face between each node and its neighbour in +axis (the
 * caller samples beta there); the face on the minus side of a node is its
 * neighbour's.  Then a_k = (sum of the regular sides' beta_face, in side
 * order) + (sum of the records' c), and a record's c is beta_face times its
 * interpolation weight (1/q or the RBF weight), so eb_assemble_rhs is
 * unchanged.  The operator's entry toward a computational neighbour is
 * -beta_face / h^2 (amg_setup_beta).  beta = 1 gives eb_assemble_diag_mode
 * bit for bit.  eb_check_spd (Sec. 2.4) assumes constant beta = 1.          */
int eb_assemble_diag_beta(const eb_grid_t* g, const double* psi, const double* beta, int32_t mode,
                          int8_t* kind, double* a, eb_cut_t* cuts, int64_t cuts_cap,
                          int64_t* n_unknowns, int64_t* n_cuts, void* stream);

/* A-priori SPD test (Sec. 2.4, Lemma 2.1, Theorems 1-2): along every axis,
 * every maximal run of computational points on a grid line is one segment of
 * the 1-D matrix D^(n)(a, b) whose end entries a, b are the part of the
 * diagonal contributed by the two sides along that axis (1 for a
 * computational neighbour, the sum of the side's records' c for a cut side).  Every segment
 * satisfying Lemma 2.1 makes the operator SPD; a failing segment does not
 * prove the contrary (the conditions are sufficient).  Rows built by the
 * line-by-line treatment always pass (Corollary 1); RBF rows (Sec. 2.2) can
 * fail, which is what Algorithm 2 runs the test for.
 *   kind  [in]  node field from eb_assemble_diag.
 *   cuts  [in]  all n_cuts records of that assembly (sorted by node, then
 *               side), possibly with altered c.
 *   n_segments, n_failing [host out] segments over all axes, and those that
 *               fail Lemma 2.1.
 * Synchronises `stream`.  EB_EINVAL when a cut side has no record or an
 * unknown sits on the outer node layer.  Deterministic (integer counts).      */
int eb_check_spd(const eb_grid_t* g, const int8_t* kind, const eb_cut_t* cuts, int64_t n_cuts,
                 int64_t* n_segments, int64_t* n_failing, void* stream);

/* Right-hand side of steps 2-3: b_k = f_k + sum over the cuts of k of
 * u_at_cuts[m] * c_m / h^2 (the g_Gamma u_Gamma / h^2 term of Sec. 2.1.1),
 * b = 0 off computational points.  f is a node field, u_at_cuts holds the
 * Dirichlet data at each record's crossing (same order as cuts).  Deterministic
 * (no atomics).                                                                */
int eb_assemble_rhs(const eb_grid_t* g, const int8_t* kind, const double* f,
                    const eb_cut_t* cuts, int64_t n_cuts, const double* u_at_cuts,
                    double* b, void* stream);

/* eb_assemble_rhs for an island canvas (several geometries stacked along the
 * last axis on a grid of spacing 1, as pcg_solve_islands takes them): island
 * k owns node rows seg_rows[k] .. seg_rows[k+1]-1 and has its own spacing
 * seg_h[k].  Its operator on the canvas is h_k^2 times its own, so its
 * equation is multiplied by h_k^2: b = h_k^2 f + sum of u c over the records
 * (the boundary terms carry 1/h^2 = 1 of the canvas).  seg_rows (nseg + 1
 * entries, from 0 to the number of node rows) and seg_h are HOST arrays.
 * Synchronises `stream`.  EB_EINVAL on bad segments or h <= 0.               */
int eb_assemble_rhs_islands(const eb_grid_t* g, const int8_t* kind, const double* f,
                            const eb_cut_t* cuts, int64_t n_cuts, const double* u_at_cuts,
                            int32_t nseg, const int32_t* seg_rows, const double* seg_h, double* b,
                            void* stream);

/* y = A x on node fields (Eq. central_difference with the diagonal above):
 * y_k = (a_k/h^2 + sigma) x_k - (1/h^2) sum of x over computational
 * neighbours; values of x off computational points are ignored; y = 0 there. */
int stencil_apply(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma,
                  const double* x, double* y, void* stream);

/* stencil_apply for the variable-conductivity operator (eb_assemble_diag_beta):
 * each computational neighbour enters with its face's beta (beta as there).  */
int stencil_apply_beta(const eb_grid_t* g, const int8_t* kind, const double* a, const double* beta, double sigma,
                       const double* x, double* y, void* stream);

/* Time-stepper right-hand sides on the same operator (node fields; outputs are
 * 0 off computational points; asynchronous).
 *
 * Wave equation u_tt = Lap u, theta-scheme (Sec. 3.5):
 *   (I + theta dt^2 A) u^{n+1} = 2 u^n - u^{n-1} - dt^2 A ((1 - 2 theta) u^n + theta u^{n-1}).
 * eb_wave_rhs writes out = scale * (right-hand side above) from un = u^n and
 * unm1 = u^{n-1}.  theta = 0 (leap-frog) with scale = 1 gives u^{n+1}
 * itself; for theta > 0, scale = sigma = 1/(theta dt^2) gives the right-hand
 * side of (A + sigma I) u^{n+1} = out, solved by pcg_solve on a hierarchy set
 * up with that sigma.  EB_EINVAL for theta < 0, dt <= 0 or a non-finite scale. */
int eb_wave_rhs(const eb_grid_t* g, const int8_t* kind, const double* a, double theta, double dt, double scale,
                const double* un, const double* unm1, double* out, void* stream);
/* The same with the variable-conductivity operator (cond: the face fields of
 * eb_assemble_diag_beta).                                                    */
int eb_wave_rhs_beta(const eb_grid_t* g, const int8_t* kind, const double* a, const double* cond, double theta,
                     double dt, double scale, const double* un, const double* unm1, double* out, void* stream);

/* out = alpha (A + sigma I) x + beta y + gamma z.  With sigma = -2/dt,
 * alpha = -1, y = b^n, z = b^{n+1} it is the right-hand side of the
 * Crank-Nicolson heat step (Sec. 3.4) (A + (2/dt) I) u^{n+1}
 * = ((2/dt) I - A) u^n + b^n + b^{n+1}.  y (z) may be null when beta (gamma)
 * is 0; EB_EINVAL otherwise.                                                   */
int eb_stencil_combine(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma, double alpha,
                       const double* x, double beta, const double* y, double gamma, const double* z, double* out,
                       void* stream);
/* The same with the variable-conductivity operator (cond as above; the
 * Crank-Nicolson step of the Sec. 3.4 example, beta = 1/4 - x^2 - y^2).     */
int eb_stencil_combine_beta(const eb_grid_t* g, const int8_t* kind, const double* a, const double* cond,
                            double sigma, double alpha, const double* x, double beta, const double* y, double gamma,
                            const double* z, double* out, void* stream);

/* Linear quantities of interest over the islands of a canvas (Sec. 3.6: the
 * value of u at a node, the integral of u over a region, as w . u with node
 * weights w).  out[j * nseg + s] = sum of w[n] x[j * field_nodes + n] over the
 * nodes n of node rows seg_rows[s] .. seg_rows[s+1] - 1 (row_len nodes a row),
 * for the nfields fields stored back to back in x.  w (field_nodes doubles)
 * and x (nfields * field_nodes doubles) are device arrays; seg_rows (nseg + 1
 * non-decreasing row indices, the last at most field_nodes / row_len) and out
 * (nfields * nseg doubles) are host arrays.  Sums are taken in a fixed order
 * (run-to-run identical).  1 <= nfields, nseg <= 65535; EB_EINVAL for null
 * pointers or segments outside the field.  Synchronises `stream`.             */
int eb_segment_dots(const double* w, const double* x, int32_t nfields, int64_t field_nodes, int64_t row_len,
                    int32_t nseg, const int32_t* seg_rows, double* out, void* stream);

/* eb_segment_dots for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops of a shape optimisation, harnesses
 * that forbid hipMalloc): the same arguments, kernels and results (bit for
 * bit), but the segment bounds, chunk partials and results live in a fixed
 * 8 MiB device array of the library, one per GPU, held until the process
 * ends; the call makes no device allocation or free.  The array must hold
 * 16 nseg + 8 nfields nseg (nchunk + 1) bytes, nchunk = ceil(longest segment
 * in nodes / 2048): EB_ENOSPC otherwise (nothing runs).  Every call on a GPU
 * uses that GPU's one array, so calls that overlap on one GPU (different
 * streams or threads) race; each call writes all of the array it reads.
 * Synchronises `stream`.                                                      */
int eb_segment_dots_noalloc(const double* w, const double* x, int32_t nfields, int64_t field_nodes,
                            int64_t row_len, int32_t nseg, const int32_t* seg_rows, double* out, void* stream);

/* Build the aggregation AMG hierarchy of A (+ sigma I) on the device
 * (Algorithm 2 step 4 preconditioner).  *H receives a new handle (host).
 * p may be NULL for defaults.  Synchronises `stream` (level sizes are read
 * back to size allocations).  All later calls on H use the stream given here
 * unless they take their own.                                                  */
int amg_setup(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma,
              const amg_params_t* p, amg_handle_t** H, void* stream);

/* amg_setup for the variable-conductivity operator of eb_assemble_diag_beta:
 * beta as there (dim face fields, device, read during the call only).  The
 * hierarchy is built from that operator; pcg_solve and the V-cycle calls
 * run the fine level with face-weighted kernels.  Not available with it:
 * batched and island solves, per-point smoother weights and the learned
 * smoother calls, and the BF16 smoother (EB_ENOTIMPL); the FP64 and FP32
 * V-cycles are.  EB_EINVAL for a null beta; otherwise as amg_setup.         */
int amg_setup_beta(const eb_grid_t* g, const int8_t* kind, const double* a, const double* beta, double sigma,
                   const amg_params_t* p, amg_handle_t** H, void* stream);

/* amg_setup for a canvas of islands (several geometries stacked one above the
 * other, as pcg_solve_islands takes them; no stencil joins two islands, so
 * every level is block diagonal over the islands).  seg_rows (host, nseg + 1
 * int32): the first node row of each island, then the node-row count.  Each
 * island's part of the hierarchy ends where its own hierarchy would (the
 * first level on which it has at most p->coarse_max unknowns, from level 1
 * on): its unknowns take no part in the coarser levels, and the V-cycle
 * solves its diagonal block of that level exactly (kept inverted, one
 * workgroup per island); the level on which the last islands end is the
 * coarsest.  The aggregation boxes of level l are 3^(l+1) node rows tall, so
 * an island must start on a node row that is a multiple of 3^l for every
 * level l on which it ends to be one contiguous row range: EB_EINVAL names
 * the island and level otherwise (stack islands at multiples of 81 for up to
 * five levels).  EB_ENOSPC if an island ends with more than 258 unknowns
 * (coarse_max above 256).  2-D, constant conductivity; otherwise as
 * amg_setup, and pcg_solve_islands / pcg_solve_batched / pcg_solve run on the
 * handle as on any other.                                                     */
int amg_setup_islands(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma, int32_t nseg,
                      const int32_t* seg_rows, const amg_params_t* p, amg_handle_t** H, void* stream);

/* Solve A x = b by PCG with one V(1,1) cycle as preconditioner (Algorithm 2
 * step 4).  b, x are node fields; x holds x0 on entry if p->x0_given.  On
 * return x holds the solution at computational points and 0 elsewhere.
 * res (host) is filled on EB_OK and on EB_ENOCONV/EB_ENOTSPD/EB_ENAN.
 * Synchronises `stream` at return.  One handle must not be used by two
 * streams at once.                                                            */
int pcg_solve(amg_handle_t* H, const double* b, double* x, const pcg_params_t* p,
              pcg_result_t* res, void* stream);

/* PCG iterations from the third on are launched as a captured HIP graph of
 * two iterations (kernel nodes only), kept on the handle per V-cycle
 * precision, unless disabled here (process-wide; 1 = on, the default).  The
 * results are the same either way: the same kernels run with the same
 * arguments in the same order.                                                */
int eb_set_iteration_graphs(int32_t enabled);

/* The same PCG for nrhs right-hand sides (1 <= nrhs <= 64) sharing the
 * hierarchy, run as one launch sequence (Algorithm 2 step 4 for several b, as
 * in the heat steps of Sec. 3.4).  b and x hold nrhs node fields back to back
 * (field j at offset j * (n[0]+1)(n[1]+1)[(n[2]+1)] doubles); x holds the
 * initial guesses if p->x0_given.  Each right-hand side has its own
 * iteration, convergence test, true-residual check and restart; res (host)
 * receives nrhs results (solve_ms is the time of the whole batch).  Returns
 * EB_OK if every right-hand side converged, else the first failure code in
 * right-hand-side order; every res[j] is filled either way.  Internally the
 * vectors interleave the right-hand sides node by node; the first call with a
 * given slot count (nrhs rounded up to a power of two) and precision makes
 * the batch buffers, kept until amg_free.  Synchronises `stream`.            */
int pcg_solve_batched(amg_handle_t* H, int32_t nrhs, const double* b, double* x, const pcg_params_t* p,
                      pcg_result_t* res, void* stream);

/* Island batch: several geometries (of different sizes) in one hierarchy and
 * one launch sequence, each with its own PCG per right-hand side.  The
 * caller places the geometries' node grids one above the other in one node
 * grid (the canvas; every island keeps its outer layer of outside nodes, so
 * no stencil couples two islands and every aggregate, coarse operator and
 * the coarsest inverse stay block diagonal) and sets the hierarchy up on it
 * with h = 1: island i then carries h_i^2 A_i, and its source enters as
 * h_i^2 f_i (boundary terms need no scaling).  seg_rows (host, nseg + 1
 * increasing values) gives the node rows of the segments: segment s is rows
 * seg_rows[s] .. seg_rows[s+1] - 1 (a row is the y index in 2-D, z * ny + y
 * in 3-D); every unknown must lie in a segment (EB_EINVAL otherwise).  b, x:
 * nrhs canvas node fields back to back; res [out, host]: nseg * nrhs results,
 * res[s * nrhs + j], each with its own stopping test ||r|| <= tol ||b||
 * restricted to its segment.  1 <= nseg <= 1024 and nseg * (nrhs rounded up
 * to a power of two) <= 4096; the hierarchy must have two or more levels
 * (EB_ENOTIMPL otherwise).  Synchronises `stream`.                          */
int pcg_solve_islands(amg_handle_t* H, int32_t nrhs, int32_t nseg, const int32_t* seg_rows, const double* b,
                      double* x, const pcg_params_t* p, pcg_result_t* res, void* stream);

/* Launch shape of the batched fine kernels (pcg_solve_batched and
 * pcg_solve_islands): the plane width (right-hand sides stored together per
 * node) and the planes one block handles.  By default an autotuner picks
 * them on the first solve with new batch buffers: every candidate (width 8
 * or 16, 1, 2 or 4 planes per block) times the two largest fine kernels on
 * the real buffers, the fastest is kept with the buffers and in a
 * process-wide table keyed by the problem shape.  pcg_batched_set_launch_shape
 * fixes the shape for batch buffers made afterwards (width 8, 16, 32 or 64;
 * 1, 2 or 4 planes per block; 0, 0 returns to the autotuner; EB_EINVAL
 * otherwise).  pcg_batched_launch_shape reports the shape in use on H and, if
 * ncand is given, the timed candidates (at most 8; host arrays; EB_EINVAL
 * before the first batched solve on H).                                       */
int pcg_batched_set_launch_shape(int32_t plane_width, int32_t planes_per_block);
int pcg_batched_launch_shape(const amg_handle_t* H, int32_t* plane_width, int32_t* planes_per_block,
                             int32_t* ncand, int32_t* cand_width, int32_t* cand_planes, float* cand_ms);

/* Apply one V(1,1) cycle z = M r (node fields; parity and debugging aid).     */
int amg_vcycle_apply(amg_handle_t* H, const double* r, double* z, void* stream);

/* The same cycle in single precision: r is rounded to FP32 after the fine
 * pre-smoothing residual is formed, every level below computes and stores
 * FP32 (the coarsest dense solve accumulates in FP64), and z is returned
 * widened to FP64.  The first call on a handle makes FP32 copies of the
 * hierarchy's values (kept until amg_free).  Synchronises `stream`.          */
int amg_vcycle_apply_fp32(amg_handle_t* H, const double* r, double* z, void* stream);

/* The cycle in the given precision (EB_PREC_FP64, EB_PREC_FP32 or
 * EB_PREC_BF16; the BF16 smoother's z is returned widened to FP64).  The
 * first BF16 call on a handle makes the BF16 copies (kept until amg_free).
 * Synchronises `stream`.  EB_EINVAL for another precision, EB_ENOTIMPL for
 * EB_PREC_BF16 while per-point smoother weights are set.                    */
int amg_vcycle_apply_prec(amg_handle_t* H, const double* r, double* z, int32_t precision, void* stream);

/* Smoothing weight of coarse level `level` (1 <= level < levels - 1; the
 * coarsest is solved exactly) in the V-cycle's pre- and post-smoothing:
 * factor times the set-up weight 4 / (3 rho) (factor 1 restores it).  The
 * smoothed prolongators built at setup keep their weight.  Used by the
 * learned smoother (per-level weights); later solves, V-cycles and batched
 * solves on H use it.  Asynchronous on `stream`; EB_EINVAL on a bad level or
 * a factor that is not finite and positive.                                 */
int amg_set_level_weight(amg_handle_t* H, int32_t level, double factor, void* stream);

/* ------------------------------------------------------------------------
 * Learned fine-level smoother (an extension of the method: the paper fixes
 * no smoother, Sec. 3 preamble / Algorithm 2 step 4).  A convolutional
 * network (3 layers, 3^d taps, 16 channels, zero padding; bfloat16 weights,
 * FP32 arithmetic) maps two node features, a_k / (2d) at computational points
 * and clip(psi / h, -3, 3) / 3, to a Jacobi weight per computational point,
 * omega_k = omega0 (1 + tanh(o_k) / 2).  The fine level's pre- and
 * post-smoothing then use omega_k / A_kk; the prolongator and the coarser
 * levels are unchanged.  Parameters: one FP32 array (see eb_smoother_net_size)
 * in the order W1 [16][2][T], b1 [16], W2 [16][16][T], b2 [16], W3 [1][16][T],
 * b3 [1], T = 3^d taps in lexicographic order, x fastest.
 * ------------------------------------------------------------------------ */

/* Number of FP32 parameters of the network for dim 2 or 3 (-1 otherwise).     */
int64_t eb_smoother_net_size(int32_t dim);

/* Forward pass over the node grid.  kind, a, psi: node fields as produced by
 * eb_assemble_diag.  z1, z2 [out]: pre-activation fields of layers 1 and 2
 * (nodes x 16 FP32, node-major, channels fastest; kept for the backward pass;
 * z1 16-byte aligned, EB_EINVAL otherwise);
 * o [out]: the last layer (nodes FP32); omega [out]: node field of the
 * weights (0 off computational points).  Asynchronous.                       */
int eb_smoother_forward(const eb_grid_t* g, const int8_t* kind, const double* a, const double* psi,
                        const float* params, double omega0, float* z1, float* z2, float* o, double* omega,
                        void* stream);

/* Gradient of a loss with respect to the parameters, given dL/domega (node
 * field; only computational points are read) and the forward pass's z1, z2,
 * o.  scratch: eb_smoother_scratch_floats(g) FP32 values of device memory,
 * 16-byte aligned (EB_EINVAL otherwise);
 * grads [out]: eb_smoother_net_size(dim) FP32 values.  Weight gradients are
 * summed in a fixed order (deterministic).  Asynchronous.                     */
int eb_smoother_backward(const eb_grid_t* g, const int8_t* kind, const double* a, const double* psi,
                         const float* params, double omega0, const float* z1, const float* z2, const float* o,
                         const double* grad_omega, float* scratch, float* grads, void* stream);
int64_t eb_smoother_scratch_floats(const eb_grid_t* g);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
 * t >= 1) on n FP32 parameters; m, v are the moment arrays (zero at t = 1).  */
int eb_adam_step(float* params, const float* grads, float* m, float* v, int64_t n, int32_t t, float lr,
                 void* stream);

/* Use per-point weights omega (node field, positive and finite at every
 * computational point; EB_EINVAL otherwise) in the fine smoother of every
 * later pcg_solve / amg_vcycle_apply(_fp32) on H, until amg_clear_fine_weights.
 * No effect on a one-level hierarchy.  Synchronises `stream`.                 */
int amg_set_fine_weights(amg_handle_t* H, const double* omega, void* stream);
int amg_clear_fine_weights(amg_handle_t* H);

/* Training samples: for each of the m node fields xi_j (back to back), apply
 * `sweeps` times e <- (e - M A e) / ||e - M A e||_2 with the current V-cycle M
 * (fine weights if set) and write e_j (node fields, 0 off computational
 * points).  Synchronises `stream`.                                            */
int amg_smoother_samples(amg_handle_t* H, int32_t m, int32_t sweeps, const double* xi, double* e, void* stream);

/* Loss L = mean_j (e_j'^T A e_j') / (2 e_j^T A e_j), e' = e - M A e, of the
 * current V-cycle (fine weights if set) on the m node fields e_j, and its
 * gradient with respect to the fine weights omega_k (node field grad_omega,
 * 0 off computational points), by the adjoint of the cycle:
 *   g = -A e' / (e^T A e), u = g - A W g, v = u - A P E_c R u,
 *   dL/domega_k = (g_k t2_k + v_k r_k) / A_kk,
 * r = A e, t2 = r - A z2, z2 the prolongated pre-smoothed iterate, E_c the
 * coarse cycle.  loss is a host pointer.  Synchronises `stream`.              */
int amg_smoother_loss_grad(amg_handle_t* H, int32_t m, const double* e, double* loss, double* grad_omega,
                           void* stream);

/* Hierarchy introspection (host calls; pointers as described above).          */
int amg_num_levels(const amg_handle_t* H);
int amg_level_info(const amg_handle_t* H, int level, amg_level_info_t* out);
/* Fine-level node list: node_of_unknown[k] = flat node index of unknown k.    */
const int64_t* amg_fine_nodes(const amg_handle_t* H);

/* Measurement hook for benchmark harnesses (host calls).  While a kernel id
 * is selected, every launch of that solve-phase kernel made through H is
 * bracketed by HIP events on the stream it is launched on.  eb_timing_read
 * synchronises that stream, returns the number of timed launches and their
 * summed duration in ms, and resets both.  kernel_id < 0 disables timing.   */
enum {
    EB_K_PCG_SPMV = 0,      /* p <- z + beta p; q = A p; (p, q)                    */
    EB_K_PCG_XR = 1,        /* x += alpha p; r -= alpha q; ||r||^2, fused with the
                               fine pre-smoothing and residual                      */
    EB_K_FINE_DOWN = 2,     /* fine pre-smoothing and residual (first V-cycle)     */
    EB_K_FINE_RESTRICT = 3, /* fine residual restriction P^T res                   */
    EB_K_FINE_UP = 4,       /* fine prolongation and correction                    */
    EB_K_FINE_POST = 5,     /* fine post-smoothing and (r, z)                      */
    EB_K_COUNT = 6
};
int eb_timing_select(amg_handle_t* H, int kernel_id);
int eb_timing_read(amg_handle_t* H, int64_t* launches, double* total_ms);

void amg_free(amg_handle_t* H);

/* The library recycles device blocks freed by amg_free and its own
 * temporaries instead of returning them to the driver.  This synchronises the
 * current device and returns every cached, unused block (host call).          */
void eb_release_cached_memory(void);
const char* eb_strerror(int code);
const char* eb_last_error(void);
int eb_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EBAMG_H */
