/*
 * hdp -- dual-primal spectral-element Helmholtz solver for MI355X (gfx950).
 *
 * C ABI of the interface-problem solver of Galagusz & McFee, "An iterative
 * domain decomposition, spectral finite element method on non-conforming
 * meshes suitable for high frequency Helmholtz problems" (arXiv:1808.04713).
 *
 * The boundary value problem is the paper's prototype PDE (Sec. 2, eqs.
 * prototype_pde and prototype_robin) with alpha = I, beta = -k^2 eps_r
 * (piecewise constant per element) and, on the whole outer boundary, the
 * first-order impedance condition d_n u - i k u = g (time factor e^{-i w t};
 * Robin coefficient gamma = -i k).  The discretisation is the paper's
 * integrated-Legendre spectral element method on axis-aligned quadtree
 * leaves (Sec. 2.1-2.2); continuity is imposed by hierarchical edge moments
 * whose first l+1 orders per edge form the primal (coarse) space and whose
 * remaining orders are dual (Sec. 2.3.2-2.3.4).  The interface system
 * C^ A^-1 C^T nu = C^ A^-1 b^ (eq. schur_complement_system) is solved by
 * left-preconditioned GMRES with the Laplace-only Dirichlet preconditioner
 * (eqs. general_preconditioner, weight_matrix).
 *
 * Conventions
 *  - Complex numbers are interleaved (re, im) doubles (hdp_c64).
 *  - Elements are the mesh leaves in the caller's order.  Element e has
 *    degree p_e and n_e = p_e + 1 modes per direction.
 *  - Fields are returned at the (n_e x n_e) tensor Gauss-Lobatto-Legendre
 *    nodes of each element, x index fastest, elements concatenated in leaf
 *    order; with several right-hand sides the field of RHS r starts at
 *    r * sum_e n_e^2 (RHS-major).
 *  - Dual vectors passed to the operator entry points use the solver's
 *    internal layout: row-major [n_lambda][n_rhs] (RHS index fastest).
 *    Dual rows are numbered edge by edge in the visiting order of the
 *    paper's Algorithm 1 (finest level first, leaves in caller order, sides
 *    left, right, bottom, top), orders k = l+1 .. max(p_a, p_b) ascending;
 *    a row reads +sqrt(2) times the neighbour's trace coefficient minus
 *    sqrt(2) times the visiting element's (eq. final_constraint in the
 *    vertex basis of eq. interpolatory_relation).
 *  - Pointers documented as "device" must be device memory of the handle's
 *    device.  A handle issues its work on a stream of its own, ordered after
 *    the work already enqueued on the caller's stream (hdp_options.stream);
 *    unless stated otherwise a call returns after that work has finished.
 *  - The caller owns every array it passes.  A handle owns its device
 *    memory.  Handles are not thread-safe; distinct handles are independent.
 *  - On an error (negative status) output arrays are left untouched and
 *    hdp_last_error_detail() describes the cause.
 */
#ifndef HDP_H
#define HDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } hdp_c64;

typedef enum {
  HDP_OK = 0,
  HDP_W_NOT_CONVERGED = 1,  /* outputs hold the last iterate */
  HDP_W_TRUE_RESIDUAL = 2,  /* the preconditioned residual reached tol but the true interface
                               residual ||g - F nu|| / ||g|| (hdp_stats.true_residual) exceeds
                               max(1e3 tol, 1e-6): the preconditioner's row scaling hides the
                               error, as with hanging-edge constraints of tiny diagonal a^k kept
                               by discard_tol = 0 (Sec. 2.2.4); outputs hold the iterate */
  HDP_E_ARG = -1,           /* invalid argument (null pointer, size, NaN) */
  HDP_E_MESH = -2,          /* leaves do not tile the domain, or unsupported topology */
  HDP_E_RESONANCE = -3,     /* an element block A_11 is (near) singular at this k */
  HDP_E_COARSE = -4,        /* coarse matrix K singular */
  HDP_E_DEVICE = -5,        /* HIP runtime error */
  HDP_E_NOMEM = -6,         /* device allocation failed */
  HDP_E_UNSUPPORTED = -7    /* valid input outside what this build implements */
} hdp_status;

enum { HDP_FP64 = 0, HDP_MIXED = 1 };

enum {
  HDP_RHS_PLANE_WAVE_TOTAL = 0,     /* total field e^{ik d.x} through impedance data g = ik(d.n-1)u */
  HDP_RHS_POINT = 1,                /* unit point source delta(x - x0) */
  HDP_RHS_PLANE_WAVE_SCATTERED = 2, /* scattered field: f = k^2 (eps_r - 1) e^{ik d.x}, g = 0 */
  HDP_RHS_ELEMENT_LOADS = 3         /* caller's element load vectors b_e (vertex basis) */
};

typedef struct {
  double x0, x1, y0, y1;      /* domain */
  int32_t base_nx, base_ny;   /* base grid; each cell roots a quadtree */
  int32_t n_leaves;
  const int32_t* leaf;        /* host, 3 per leaf: level, ix, iy (ix,iy on that level's grid) */
  const int32_t* degree;      /* host, p per leaf, 1 <= p <= 40 */
} hdp_mesh;

typedef struct {
  double k;                   /* free-space wavenumber, > 0 */
  const double* eps_r;        /* host, per leaf relative permittivity; NULL means 1 */
  int32_t l;                  /* coarse order; <= 0 selects the dispersion rule (Sec. 2.3.4),
                                 evaluated with each element's longest edge and local
                                 wavenumber k sqrt(eps_r) (or k, l_free_space), the largest
                                 value taken */
  int32_t l_safety;           /* added to the rule's value (the paper adds 1 in Sec. 3.3) */
  double discard_tol;         /* Sec. 2.2.4: a dual constraint of degree k on the fine side of
                                 a hanging edge is dropped when the diagonal a^k of its change
                                 of basis L_c^f is below this value (0 keeps every constraint;
                                 primal constraints are always kept) */
  int32_t robin_modified;     /* Sec. 2.3.4: 1 adds Robin terms gamma = +-ik to the local
                                 problems on the interior sides between elements of opposite
                                 label (breadth-first levels from leaf 0, neighbours taken side
                                 by side, left right bottom top, and across one side in leaf
                                 order; even levels +ik, odd -ik).  The terms cancel in the
                                 assembled system, so the solution is unchanged, while every
                                 local problem becomes uniquely solvable at element resonances.
                                 HDP_E_UNSUPPORTED when a side's neighbours carry both labels
                                 (possible on hanging sides).  0: unmodified. */
  const double* pml_sigma;    /* Sec. 3.3: host, 2 per leaf (sigma_x, sigma_y) >= 0, or NULL for
                                 none.  Axis-aligned perfectly matched layers by complex
                                 stretching s = 1 + i sigma / k (e^{-i omega t}, omega = k):
                                 alpha = diag(s_y/s_x, s_x/s_y), beta = -k^2 eps_r s_x s_y on the
                                 leaf; the preconditioner's Laplace part takes the same alpha.
                                 Loads stay those of the unstretched problem (a layer leaf with
                                 eps_r = 1 carries no scattered-field source).  HDP_E_UNSUPPORTED
                                 with hanging edges. */
  int32_t l_per_edge;         /* with l <= 0: 1 evaluates the dispersion rule edge by edge (the
                                 non-uniform l the conclusions propose for non-uniformly refined
                                 meshes): on each edge, for every leaf touching it, its own side
                                 length along the edge and k sqrt(eps_r), the largest value taken
                                 (plus l_safety); a hanging edge is the coarse side with its fine
                                 leaves, so both sides agree.  hdp_stats.l reports the largest. */
  int32_t l_free_space;       /* with l <= 0: 1 evaluates the dispersion rule with the free-space k
                                 instead of the local k sqrt(eps_r) (the reading of the paper's
                                 dielectric-cylinder example, Sec. 3.3.1, where h is the longest
                                 edge); 0 (default) takes the local wavenumber, which keeps the
                                 iteration count low inside dielectrics (the free-space rule
                                 leaves the coarse problem under-resolved there: 8 against 59
                                 iterations on a 10x10 mesh with an eps_r = 4 block at k = 25). */
} hdp_problem;

/* Device memory of a handle: hipMalloc / hipFree unless the caller passes its own
 * pair (a framework's caching allocator, a memory pool).  alloc(bytes, ctx) returns
 * memory of the current device, aligned to at least 256 bytes, or NULL (the call
 * that needed it then fails with HDP_E_NOMEM); free(p, ctx) takes back a block alloc
 * returned.  hdp_destroy, and a failing hdp_setup, free every block the handle took
 * after its stream has finished.  Both pointers set, or both NULL. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* p, void* ctx);
  void* ctx;
} hdp_allocator;

typedef struct {
  int32_t precision;          /* HDP_FP64, or HDP_MIXED (FP32 local operators, FP64 outer GMRES) */
  double tol;                 /* preconditioned relative residual target, e.g. 1e-8 */
  int32_t max_iter;           /* GMRES iteration cap (no restart), 1..1000 */
  int32_t max_rhs;            /* largest n_rhs that hdp_solve will receive, 1..64 */
  void* stream;               /* caller's hipStream_t (NULL: null stream) the solver orders after */
  int32_t flags;              /* HDP_FLAG_* bits, 0 for defaults */
  int32_t tile_fdm;           /* right-hand sides per workgroup of the separable element solve on
                                 the matrix cores (1, 2, 4, 8 or 16; 0: the autotuner's choice
                                 with HDP_FLAG_AUTOTUNE, else a shared-memory heuristic) */
  int32_t tile_slot;          /* right-hand sides per workgroup of the matrix-core slot operators
                                 at 16 or more columns (16, 32 or 64; 0: autotuned or 32) */
  hdp_allocator allocator;    /* device memory of the handle (zero: hipMalloc / hipFree) */
} hdp_options;

/* hdp_options.flags: replay each GMRES iteration as a captured HIP graph
 * instead of launching its kernels one by one. */
#define HDP_FLAG_GRAPH 1
/* coarse factor: by default a dense inverse up to 6,000 coarse unknowns and the
   nested-dissection multifrontal factor above; these flags force one of them (at most
   one may be set).  When the set-up check of the factor (hdp_stats.coarse_residual)
   exceeds 1e-10, every coarse solve is refined once against the assembled K (the
   check reports the refined solve).  HDP_FLAG_COARSE_BLOCK named a block-tridiagonal
   strip factor that is no longer provided: setting it is HDP_E_ARG. */
#define HDP_FLAG_COARSE_BLOCK 2
#define HDP_FLAG_COARSE_DENSE 4
#define HDP_FLAG_COARSE_ND 8
/* time every candidate tile width of the separable element solve and of the
   matrix-core slot operators, and (nested-dissection coarse factor, max_rhs > 1)
   every split target of the coarse sweeps, at set-up, on the handle's own mesh
   at max_rhs columns, and keep the fastest (hdp_autotune_table lists the
   measurements); tile_fdm / tile_slot, when non-zero, take precedence */
#define HDP_FLAG_AUTOTUNE 16

typedef struct {
  int32_t kind;               /* HDP_RHS_* */
  int32_t n_rhs;              /* 1 .. max_rhs */
  const double* angles;       /* host, n_rhs propagation angles (plane-wave kinds) */
  const double* points;       /* host, 2*n_rhs source points (HDP_RHS_POINT) */
  const hdp_c64* loads;       /* device, dof * n_rhs values, [dof][n_rhs] (RHS index fastest):
                                 per leaf the (p+1)^2 coefficients of int N~_a N~_b f + boundary
                                 terms in the vertex basis, x index fastest (HDP_RHS_ELEMENT_LOADS) */
} hdp_rhs;

typedef struct {
  int64_t dof;                /* sum_e n_e^2 */
  int32_t n_elements, n_lambda, n_coarse, l, n_classes;
  int32_t iterations;         /* GMRES iterations (max over RHS; mixed: inner iterations in total) */
  int32_t refinements;        /* outer refinement steps (mixed precision), else 0 */
  double rel_residual;        /* final preconditioned relative residual, max over RHS */
  double min_element_margin;  /* min over element classes of min|lambda_x+lambda_y| / max|.| */
  double setup_ms, solve_ms;
  /* host-side breakdown of solve_ms: loads and interface right-hand side,
   * GMRES (launch calls, waits for the device), recovery and sampling */
  double rhs_ms, gmres_ms, gmres_launch_ms, gmres_wait_ms, recover_ms;
  double true_residual;       /* ||g - F nu|| / ||g|| in FP64 after the solve, max over RHS */
  double coarse_residual;     /* setup check of the coarse factor: ||K x - b|| / ||b|| */
  int32_t coarse_mode;        /* 0 dense inverse, 2 nested dissection */
  int32_t coarse_blocks;      /* nested-dissection tree nodes (1 for the dense inverse) */
  double coarse_factor_bytes; /* bytes of the coarse factor as stored (dense inverse or
                                 nested-dissection fronts) */
  double coarse_band_bytes;   /* bytes of a banded (envelope) LU factor of K with the coarse unknowns
                                 in breadth-first level order (bandwidth-reducing, from the bottom
                                 edge): what one coarse solve with a plain factorisation reads */
  /* set-up breakdown (host wall clock, ms): the host analysis as a whole (constraints,
   * element classes, coarse maps), its element-class operators (eigenbases, unit solves,
   * Schur blocks; built on up to 16 host threads), and the coarse factor */
  double setup_host_ms, setup_classes_ms, setup_coarse_ms;
  /* nested-dissection factor at several columns: the unknowns of the tree's top
   * depths solved as one dense block (rows of K^-1 at those unknowns, built at
   * set-up), 0 when the sweeps run every depth; and the set-up check of the sweeps
   * with the block, ||K x - b|| / ||b|| over two columns (the block is not used
   * when it exceeds max(1e-10, 10 coarse_residual)) */
  int32_t coarse_top_unknowns;
  double coarse_top_check;
} hdp_stats;

typedef struct hdp_handle hdp_handle;

/* Build the solver (paper Sec. 2.3.2-2.3.3): find conforming and hanging
 * sides (Sec. 2.2.4, any number of hanging nodes per side), classify leaves
 * into element classes, compute each class's separable eigenbasis and
 * boundary operators, number dual rows and coarse unknowns (Algorithm 1),
 * assemble the coarse matrix K = A_22 - A_12^T A_11^-1 A_12 and factor it in
 * FP64: by default a dense inverse up to 6,000 coarse unknowns and a
 * nested-dissection multifrontal factor above (fronts factored on the host,
 * sweeps on the device); HDP_FLAG_COARSE_DENSE / _ND select one of them.
 * Every coarse solve runs in the library's own kernels (a streamed symmetric
 * inverse or tile products of the inverse; the nested-dissection sweeps).
 * Leaves must tile the domain
 * (HDP_E_MESH otherwise). */
hdp_status hdp_setup(const hdp_mesh* mesh, const hdp_problem* prob,
                     const hdp_options* opt, hdp_handle** out);

/* Far-field intensity J = |E_far(far_angle)|^2 of the scattered field for the
 * plane wave of propagation angle `incidence` (HDP_RHS_PLANE_WAVE_SCATTERED),
 * and its gradient dJ/d eps_r,e for every leaf: the adjoint solve A lambda = g
 * with g = dE_far/dphi reuses the same solver (the system is complex
 * symmetric, Sec. 2.3.4), then per leaf
 *   dJ/d eps_e = 2 Re( conj(E) lambda_e^T (db_e/d eps_e - dA_e/d eps_e phi_e) ),
 * dA_e/d eps_e = -k^2 (h_x h_y / 4) M~ (x) M~, db_e/d eps_e = k^2 int N~ e^{ik d.x}.
 * far_inside: host, one byte per leaf (the region whose boundary carries the
 * far-field integral; its outside leaves give the traces).  J: host, 1 value;
 * grad: host, n_leaves values.  stats (optional) describe the forward solve.
 * Needs max_rhs >= 1; returns HDP_W_NOT_CONVERGED if a solve missed tol, or
 * HDP_W_TRUE_RESIDUAL as hdp_solve. */
hdp_status hdp_far_intensity_gradient(hdp_handle* h, double incidence, double far_angle,
                                      const uint8_t* far_inside, double* J, double* grad,
                                      hdp_stats* stats);

/* Solve for n_rhs right-hand sides at once (paper Sec. 2.3.1: interface
 * right-hand side, GMRES on the interface problem, recovery of phi).
 * field: device, n_rhs * dof complex values at GLL nodes (RHS-major), or NULL.
 * far:   device, n_rhs * n_far complex values E_far(phi_q) (Sec. 3.3.1, for the
 *        e^{-i w t} convention) over the boundary of the leaves with
 *        far_inside[e] != 0, or NULL.  far_angles: host, n_far observation
 *        angles.  far_inside: host, one byte per leaf.
 * Returns HDP_W_NOT_CONVERGED if some RHS did not reach tol in max_iter, else
 * HDP_W_TRUE_RESIDUAL if some RHS's true interface residual exceeds
 * max(1e3 tol, 1e-6). */
hdp_status hdp_solve(hdp_handle* h, const hdp_rhs* rhs, hdp_c64* field,
                     int32_t n_far, const double* far_angles, const uint8_t* far_inside,
                     hdp_c64* far, hdp_stats* stats);

/* u = F v with F = C^ A^-1 C^T (eq. schur_complement_system, conforming form
 * C_1 [A_11^-1 + A_11^-1 A_12 K^-1 A_12^T A_11^-1] C_1^T).  v, u: device,
 * [n_lambda][n_rhs] complex.  precision selects FP64 or FP32 local operators. */
hdp_status hdp_apply_interface(hdp_handle* h, const hdp_c64* v, hdp_c64* u,
                               int32_t n_rhs, int32_t precision);

/* u = P^-1 v with the Dirichlet preconditioner built from the Laplace-only
 * part (eq. general_preconditioner with W_1 of eq. weight_matrix).  On a
 * conforming mesh C_2 = 0 and P^-1 = X^-1 C_1 S_e C_1^T X^-1 with X = C_1 C_1^T;
 * with hanging edges W_2 = I, the cross term is dropped and C_2 K_L C_2^T kept
 * (the remark after the preconditioner): X = C_1 C_1^T + C_2 C_2^T (dense
 * blocks on the rows C_2 couples) and Y = C_1 S_e C_1^T + C_2 K_L C_2^T.
 * Layout as hdp_apply_interface. */
hdp_status hdp_apply_precond(hdp_handle* h, const hdp_c64* v, hdp_c64* u,
                             int32_t n_rhs, int32_t precision);

/* Allocation-free variant of hdp_apply_precond, for callers that cannot
 * allocate device memory during the call (tight serving loops, code that must
 * not call hipMalloc).  Same operation, arguments, layout and result as
 * hdp_apply_precond; the work buffers (slot values, and on meshes with hanging
 * edges the intermediate dual vectors; FP32 copies in the mixed precision) come
 * from one fixed 32 MiB array per device that the library holds until the
 * process ends, resolved at hdp_setup.  The call allocates nothing and creates
 * no profiling events (hdp_profile does not see it).
 * Limit: the work buffers must fit 32 MiB, about 16 n_rhs (n_slots + 2 n_lambda)
 * bytes; larger requests return HDP_E_ARG with the needed size in
 * hdp_last_error_detail().  Every call on one GPU shares that GPU's array (it
 * keeps the last call's contents; nothing in it needs to start at zero), so
 * calls that overlap in time on one GPU, from any handles or threads, race:
 * callers must serialise them. */
hdp_status hdp_apply_precond_noalloc(hdp_handle* h, const hdp_c64* v, hdp_c64* u,
                                     int32_t n_rhs, int32_t precision);

/* g = C^ A^-1 b^ (the interface right-hand side) for the given RHS.
 * g: device, [n_lambda][n_rhs]. */
hdp_status hdp_interface_rhs(hdp_handle* h, const hdp_rhs* rhs, hdp_c64* g);

/* x_e = A_e^-1 y_e for every element by the separable fast solver
 * X = E_x [(E_x^T Y E_y) ./ (lambda_x,i + lambda_y,j)] E_y^T (Sec. 2.2.1 remark
 * on the fast solver), on the full element matrix in the vertex basis of
 * eq. interpolatory_relation.  y, x: device, [sum_e n_e^2][n_rhs] complex,
 * element blocks in leaf order, x-mode fastest inside a block. */
hdp_status hdp_local_solve(hdp_handle* h, const hdp_c64* y, hdp_c64* x, int32_t n_rhs);

/* Host-only analysis of a problem without touching the device: sizes, l,
 * number of element classes and the smallest separable-solver margin
 * min|lambda_x + lambda_y| / max|lambda_x + lambda_y| over classes (an
 * element resonance, Sec. 2.3.4, drives it to zero). */
hdp_status hdp_inspect(const hdp_mesh* mesh, const hdp_problem* prob, hdp_stats* stats);

/* Sizes of the handle's problem (host call, no device work). */
hdp_status hdp_get_stats(const hdp_handle* h, hdp_stats* stats);

/* Preconditioned relative residual ||P^-1 r_k|| / ||P^-1 r_0|| after each
 * iteration k = 0, 1, .. of the last GMRES run of the handle, for right-hand
 * side `rhs` (the quantity plotted in the paper's residual figures, Sec. 3.2).
 * Mixed precision: the last inner run.  count receives the number of entries;
 * at most max are written to out (host). */
hdp_status hdp_residual_history(const hdp_handle* h, int32_t rhs, double* out, int32_t max, int32_t* count);

/* Kernel timing.  While enabled, every kernel launch family of the handle is
 * bracketed by HIP events on the handle's stream; hdp_profile_read returns,
 * per family, the launches, the summed event durations and the algorithmic
 * HBM bytes and floating-point operations of those launches (sizes of the
 * operands each launch must read and write once, and the useful arithmetic).
 * enable = 1 clears and starts, 0 stops.  Profiling adds per-launch event
 * overhead and is meant for measurement runs. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double bytes;
  double flops;
} hdp_kernel_time;
hdp_status hdp_profile(hdp_handle* h, int32_t enable);
hdp_status hdp_profile_read(const hdp_handle* h, hdp_kernel_time* out, int32_t max, int32_t* count);

/* The set-up autotuner's measurements (HDP_FLAG_AUTOTUNE): one entry per
 * candidate, the kernel family ("fdm_element_solve", "slot_operator",
 * "coarse_nd_split"), the candidate's parameter (right-hand sides per workgroup;
 * for coarse_nd_split the workgroups each split tree depth aims at), its mean
 * time over three launches at max_rhs columns (ms; one coarse solve for
 * coarse_nd_split) and whether it was chosen.  count receives the number of
 * entries; at most max are written to out (host). */
typedef struct {
  char kernel[32];
  int32_t cols;
  int32_t chosen;
  double ms;
} hdp_tune_entry;
hdp_status hdp_autotune_table(const hdp_handle* h, hdp_tune_entry* out, int32_t max, int32_t* count);

void hdp_destroy(hdp_handle* h);
const char* hdp_status_string(hdp_status s);
const char* hdp_last_error_detail(void);   /* thread-local, valid until the next call */

#ifdef __cplusplus
}
#endif
#endif
