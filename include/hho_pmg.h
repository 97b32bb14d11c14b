/*
 * hho_pmg.h -- C ABI of the MI355X p-multilevel HHO Stokes library.
 *
 * The library solves the Stokes problem (Section 1 of Botti & Di Pietro,
 * "p-Multilevel preconditioners for HHO discretizations of the Stokes
 * equations with static condensation", arXiv 2009.13840) with the equal-order
 * HHO scheme with discontinuous pressure (Scheme 1, Section 2.3.1), condenses
 * it cell by cell (Section 4.1.2: v-cond, eq. ST.1, or v&p-cond, eq. ST.2),
 * inherits coarse operators of degrees k_0 > k_1 > ... > k_L by Galerkin
 * projection of the condensed operator (Sections 3.2 and 4.2), and solves it
 * with flexible GMRES preconditioned by one p-multilevel V-cycle per
 * iteration (algorithm of Section 3.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status: HHO_OK (0) or a negative HHO_E_*
 *   code.  No C++ exception crosses the ABI.  hho_last_error() returns a
 *   thread-local message describing the last failure.
 * - Handles are opaque.  A handle is not thread-safe: calls on one handle
 *   must be serialised by the caller.  Destroy functions accept NULL.
 * - Host pointers are read during the call only; the library copies what it
 *   keeps.  Device pointers (marked "device") must point to memory of the
 *   current HIP device; the library never frees caller memory.
 * - Device memory: after hho_problem_set_data the caller queries
 *   hho_workspace_size() and binds one device buffer of at least that many
 *   bytes with hho_bind_workspace(); every device array of the problem is
 *   carved out of it, so the library performs no device allocation of its own
 *   in setup or solve.  The buffer must stay alive until the problem is
 *   destroyed or rebound.
 * - Streams: all device work is enqueued on the stream given by
 *   hho_set_stream() (default: the null stream).  Functions that return
 *   host results synchronise that stream before returning.
 *
 * Global unknown layout ("global layout", used by every vector argument)
 * ----------------------------------------------------------------------
 * level l has degree k_l, n_F = dim P^{k_l}_{d-1}, and
 *   n_P = dim P^{k_l}_d (v-cond) or 1 (v&p-cond):
 *   face velocity  (face f, component c, mode j) -> (f*d + c)*n_F + j
 *   cell pressure  (cell T, mode q)              -> n_faces*d*n_F + T*n_P + q
 * Face modes are coefficients in the L2(F)-orthonormal hierarchical basis
 * obtained by Gram-Schmidt (twice, modified) of the scaled monomials
 * ((x - x_F).t_i / h_F)^beta in graded order, where the tangent t_1 points from
 * the face's first to its second vertex (d=3: t_2 = n_F x t_1 with n_F the
 * Newell normal of the vertex ring; d=2: n_F = (t_1y, -t_1x)).  Cell modes use
 * the L2(T)-orthonormal hierarchical basis from ((x - x_T)/h_T)^alpha
 * (x_T centroid, h_T diameter) in graded order, so the first pressure mode is
 * the mean (|T|^{-1/2}).
 */
#ifndef HHO_PMG_H
#define HHO_PMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HHO_OK                 0
#define HHO_E_INVALID_ARG     -1  /* bad argument, size or call order            */
#define HHO_E_MESH            -2  /* inconsistent mesh topology or geometry      */
#define HHO_E_LOCAL_SINGULAR  -3  /* a local Cholesky factorisation failed       */
#define HHO_E_NOT_CONVERGED   -4  /* max iterations reached; outputs are written */
#define HHO_E_BREAKDOWN       -5  /* NaN/Inf met in the iteration                */
#define HHO_E_DEVICE          -6  /* HIP runtime error (message has the code)    */
#define HHO_E_CAPACITY        -7  /* caller buffer too small                     */
#define HHO_E_OOM             -8  /* host allocation failed                      */

/* condensation variants, Section 4.1.2 */
#define HHO_COND_V   1   /* v-cond: cell velocities eliminated (eq. ST.1)              */
#define HHO_COND_VP  2   /* v&p-cond: cell velocities and non-mean pressures (eq. ST.2) */

/* precision of the V-cycle (the outer FGMRES is always FP64) */
#define HHO_PREC_FP64   0
#define HHO_PREC_FP32   1   /* levels above the coarsest: FP32 values, vectors and arithmetic */
#define HHO_PREC_BF16   2   /* levels above the coarsest: operator values stored as bfloat16
                               (rounded to nearest even from FP32), smoother factors FP32,
                               FP32 vectors and arithmetic */

/* coarsest-level solver */
#define HHO_COARSE_AUTO   0   /* DENSE up to 1024 unknowns (single problems); else, when
                                 k_L = 0, DIRECT when its fronts fit (32 GiB of fronts, the
                                 largest within one compute unit's LDS) and AMG otherwise;
                                 else GMRES                                                   */
#define HHO_COARSE_DENSE  1   /* bordered dense inverse (FP64)                                */
#define HHO_COARSE_GMRES  2   /* GMRES to coarse_rtol, cell-patch Schwarz preconditioner      */
#define HHO_COARSE_AMG    3   /* GMRES to coarse_rtol, block-triangular Stokes preconditioner
                                 with a smoothed-aggregation velocity block (k_L = 0 only)     */
#define HHO_COARSE_DIRECT 4   /* sparse direct solve (Section 5.2: the 2D coarse solver is a
                                 direct factorisation): multifrontal elimination in a nested
                                 dissection order, factorised at setup (k_L = 0 only; in a
                                 batch one pinned pressure per member with a null space)       */

/* how the face blocks of the V-cycle's level-0 copy are formed (FP32/BF16 V-cycles) */
#define HHO_COPY_CONVERT  0   /* the FP64 operator rounded to the copy's precision */
#define HHO_COPY_PRODUCT  1   /* each cell's Schur complement formed again from its FP64 factors,
                                 rounded to bfloat16 and multiplied on the matrix cores with
                                 FP32 accumulation (couplings and coarser levels: rounded) */

/* smoother preconditioner of the V-cycle's GMRES(smooth_its) steps (Section 3.3) */
#define HHO_SMOOTHER_SCHWARZ  0   /* cell-patch additive Schwarz (default) */
#define HHO_SMOOTHER_ILU      1   /* the paper's (Section 3.3): zero-fill ILU of the level operator in the
                                     natural ordering of its unknowns, exact, level-scheduled; FP64 V-cycle
                                     only, no learned smoother; also preconditions the coarse GMRES
                                     when the coarsest level is solved by it (coarse_mode GMRES) */

/* treatment of the constant-pressure null space */
#define HHO_NULLSPACE_AUTO  0   /* projected out when the boundary has no Neumann face */
#define HHO_NULLSPACE_NONE  1   /* never projected (the caller's right-hand side must be consistent) */

/* where the local operators of Sections 2.2-2.3 are built (hho_problem_set_data) */
#define HHO_LOCAL_AUTO    0   /* on the device when its limits hold (a cell's velocity unknowns d*nloc <= 1024,
                                 its work arrays within the LDS), on the host otherwise */
#define HHO_LOCAL_HOST    1   /* on the host, at hho_problem_set_data */
#define HHO_LOCAL_DEVICE  2   /* on the device, at hho_setup; set_data fails if the limits do not hold */

/* face boundary flags in hho_mesh_desc.face_bc */
#define HHO_FACE_INTERIOR   0
#define HHO_FACE_DIRICHLET  1
#define HHO_FACE_NEUMANN    2

typedef struct hho_mesh hho_mesh;
typedef struct hho_problem hho_problem;

/* Polytopal mesh (Section 2.1) in CSR form.  d=2: faces are segments given by
 * two vertices, cells are convex polygons listing their faces; d=3: faces are
 * planar convex polygons (vertex ring), cells convex polyhedra.  All arrays are
 * host memory and are copied. */
typedef struct {
  int32_t dim;                 /* 2 or 3 */
  int64_t n_verts;
  const double *verts;         /* [n_verts*dim] */
  int64_t n_faces;
  const int64_t *face_ptr;     /* [n_faces+1] */
  const int64_t *face_vtx;     /* [face_ptr[n_faces]] */
  int64_t n_cells;
  const int64_t *cell_ptr;     /* [n_cells+1] */
  const int64_t *cell_face;    /* [cell_ptr[n_cells]] */
  const int8_t *face_bc;       /* [n_faces] HHO_FACE_* ; boundary faces must be 1 or 2 */
} hho_mesh_desc;

/* Solver options; hho_options_default() fills the defaults noted here. */
typedef struct {
  double eta;          /* Nitsche penalty of eq. HHOdiscrMNT; <= 0: 4(k+1)(k+d)/d * max card(F_T) */
  double rtol;         /* FGMRES true relative residual (1e-8) */
  int32_t max_it;      /* FGMRES iterations (1000) */
  int32_t restart;     /* FGMRES restart length (30, at most 64) */
  int32_t smooth_its;  /* GMRES iterations per pre/post smoothing (2, at most 2) */
  int32_t precision;   /* HHO_PREC_* (FP64) */
  int32_t coarse_mode; /* HHO_COARSE_* (AUTO) */
  double coarse_rtol;  /* coarse GMRES relative residual (0: 1e-3 in 3D, 1e-2 in 2D) */
  int32_t coarse_restart; /* coarse GMRES restart (30, at most 64) */
  int32_t coarse_max_it;  /* coarse GMRES iterations (300) */
  int32_t quad_extra;  /* quadrature exact to degree 2k+2+quad_extra (6) */
  int32_t coarse_amg_sweeps; /* damped-Jacobi sweeps before/after the AMG coarse correction (1; 1 or 2) */
  int32_t learned;     /* 1: reserve the learned fine-level smoother (hho_learned_*); 0 (default): no */
  int32_t coarse_amg_explicit; /* AMG levels with at most this many rows are applied as the explicit
                                  matrix of their V-cycle, formed at setup (2048; 0 = never; at most 4096) */
  int32_t coarse_amg_psmooth;  /* AMG prolongator smoothing steps, at most: P = (I - w D^-1 A)^s T (1; 1 or 2;
                                  a level takes one step where two would make the next operator too dense) */
  int32_t smoother;    /* HHO_SMOOTHER_* (SCHWARZ) */
  int32_t nullspace;   /* HHO_NULLSPACE_* (AUTO) */
  int32_t vcycle_copy; /* HHO_COPY_* (CONVERT); PRODUCT needs precision FP32 or BF16 */
  int32_t local_build; /* HHO_LOCAL_* (AUTO): with the device build, hho_problem_set_data only
                          integrates the data (the callbacks run there) and hho_setup builds every
                          cell's operators on the device before the condensation */
} hho_options;

/* Scalar or vector field evaluated at n points x [n*dim]; nrm [n*dim] holds the
 * outward unit normals for boundary data (NULL for the body force).  Writes
 * out [n*dim]. */
typedef void (*hho_field_fn)(const double *x, int64_t n, const double *nrm, double *out, void *ctx);

const char *hho_last_error(void);
void hho_options_default(hho_options *opt);

/* Validates and copies a mesh: every face belongs to one or two cells, boundary
 * faces carry a Dirichlet or Neumann flag, interior faces flag 0, cells have
 * positive measure.  Errors: HHO_E_INVALID_ARG, HHO_E_MESH. */
int hho_mesh_create(const hho_mesh_desc *desc, hho_mesh **out);
void hho_mesh_destroy(hho_mesh *m);

/* Creates a problem on a mesh: degree k >= 0 (k <= 6), cond = HHO_COND_V|VP,
 * nlev levels of strictly decreasing degrees[] with degrees[0] = k
 * (degrees = NULL: k, k-1, ..., 0).  The mesh must outlive the problem.
 * Errors: HHO_E_INVALID_ARG. */
int hho_problem_create(const hho_mesh *mesh, int k, int cond, int nlev, const int *degrees,
                       const hho_options *opt, hho_problem **out);
void hho_problem_destroy(hho_problem *p);

/* Builds the local HHO operators of every cell on the host (Sections 2.2,
 * 2.3.1): potential reconstruction, face residual stabilisation, Nitsche terms,
 * pressure-velocity coupling and data terms.  f is the body force; gD the
 * Dirichlet datum; gN the traction (grad u - p I)n on Neumann faces (may be NULL
 * when there is none; NULL f/gD mean zero).  Errors: HHO_E_INVALID_ARG,
 * HHO_E_LOCAL_SINGULAR (reconstruction matrix not SPD). */
int hho_problem_set_data(hho_problem *p, hho_field_fn f, hho_field_fn gD, hho_field_fn gN, void *ctx);

/* enable = 1: every V-cycle of hho_solve (and of the calls that apply it) is
 * replayed from a HIP graph captured at its first use (captured again after
 * hho_bind_workspace or a change of precision, smoothing steps, learned
 * smoother or coarse limits).  Inside the graph the coarse GMRES takes at most
 * min(coarse_restart, coarse_max_it) columns per V-cycle with no restart and
 * tests convergence on the device, so the host issues one launch per V-cycle
 * and reads nothing during it; while the eager coarse solve needs no restart,
 * both give the same iterates.  enable = 0 (default): eager launches.  The
 * graph reads the workspace, so hho_setup with new data keeps it valid; the
 * coarse iteration count of hho_get_timings omits the captured iterations. */
int hho_set_graph(hho_problem *p, int enable);

/* Right-hand sides given directly as moments, replacing the data terms that
 * hho_problem_set_data integrated (for instance moments computed elsewhere in
 * the library's bases).  Per cell T, in mesh order: rhs_u holds d*nloc_T values,
 * component c then local unknown i at c*nloc_T + i, the local unknowns being the
 * n_T cell modes followed by the n_F modes of each face of T in T's face order
 * (nloc_T = n_T + card(F_T) n_F); rhs_p holds n_T values per cell: the
 * momentum and mass right-hand sides of the local problem of Section 2.3.1
 * (data terms of eq. def:HHOAB, with the Dirichlet datum loading cell rows as
 * well).  The local operators stay; the next hho_setup copies the records
 * again (with the device build, writes these moments over the ones it forms).
 * Needs hho_problem_set_data first (NULL fields build the operators with zero
 * data).  hho_moments_size gives the two lengths. */
int hho_moments_size(const hho_problem *p, int64_t *n_u, int64_t *n_p);
int hho_set_moments(hho_problem *p, const double *rhs_u, const double *rhs_p);

/* Device workspace (see conventions).  hho_bind_workspace fails with
 * HHO_E_CAPACITY if bytes < hho_workspace_size(). */
int hho_workspace_size(const hho_problem *p, size_t *bytes);
int hho_bind_workspace(hho_problem *p, void *dev_ptr, size_t bytes);
int hho_set_stream(hho_problem *p, void *hip_stream);

/* Copies the mesh topology and the local operators to the bound workspace
 * (host -> device).  hho_setup calls it when it has not been called; calling it
 * first keeps the transfer out of a timed setup.  Errors: HHO_E_INVALID_ARG,
 * HHO_E_DEVICE. */
int hho_upload(hho_problem *p);

/* Device setup: copies the local operators to the device, condenses every cell
 * (eq. ST.1 or ST.2, FP64 Cholesky of the local blocks), assembles the face-block
 * sparse operator, inherits the coarse levels by sub-block extraction
 * (Section 4.2), and factorises the smoother patches and the coarse solver.
 * Errors: HHO_E_INVALID_ARG (no data / workspace), HHO_E_LOCAL_SINGULAR,
 * HHO_E_DEVICE. */
int hho_setup(hho_problem *p);

/* Number of unknowns of level l in the global layout. */
int hho_level_size(const hho_problem *p, int level, int64_t *n);

/* FGMRES + V-cycle solve from x = 0 (Section 3.3), outputs in caller-owned
 * host buffers: face_out [face_n] the face velocity modes in the global layout
 * (face f, component c, mode j at (f*d + c)*n_F + j), cell_p_out [p_n] the cell
 * pressure modes kept by the condensation (cell T, mode q at T*n_P + q: every
 * mode of P^k for v-cond, the mean for v&p-cond), with face_n, p_n from
 * hho_solution_sizes; the pressure has zero mean when the boundary is all
 * Dirichlet.  iters receives the iteration count; hist (may be NULL) receives
 * min(hist_cap, iters+1) relative residual estimates, hist[0] = 1; final_rel
 * (may be NULL) the explicitly recomputed true relative residual.
 * Errors: HHO_E_CAPACITY (face_cap < face_n or p_cap < p_n; nothing solved),
 * HHO_E_NOT_CONVERGED (outputs written), HHO_E_BREAKDOWN, HHO_E_DEVICE. */
int hho_solve(hho_problem *p, double *face_out, int64_t face_cap, double *cell_p_out, int64_t p_cap, int *iters,
              double *hist, int hist_cap, double *final_rel);

/* Sizes of hho_solve's outputs: face_n = n_faces*d*n_F, p_n = n_cells*n_P (level 0). */
int hho_solution_sizes(const hho_problem *p, int64_t *face_n, int64_t *p_n);

/* hho_solve with the whole level-0 solution written to x_dev (device,
 * [level-0 size], global layout: face part then pressure part) on the problem's
 * stream instead of host buffers. */
int hho_solve_device(hho_problem *p, double *x_dev, int *iters, double *hist, int hist_cap, double *final_rel);

/* Changes the stopping rules of later hho_solve calls (options.rtol, max_it,
 * coarse_rtol, coarse_max_it; the restart lengths size the workspace and stay).
 * Errors: HHO_E_INVALID_ARG (rtol or coarse_rtol outside (0, 1), limits < 1). */
int hho_set_tolerances(hho_problem *p, double rtol, int max_it, double coarse_rtol, int coarse_max_it);

/* Back-substitution of the cell unknowns eliminated by static condensation
 * (Section 4.1.2): from the level-0 solution x_dev of hho_solve (device, global
 * layout), cell_u_dev [n_cells x d*n_T] receives the cell velocity modes
 * (component c, mode j at c*n_T + j), from the first block row of eq. def:HHOAB
 * for v-cond; cell_p_dev [n_cells x n_T] the full cell pressure modes: for v-cond
 * a copy of x's, for v&p-cond the kept mean mode and the non-mean modes from the
 * eliminated block of eq. ST.2.  Device buffers, owned by the caller, on the
 * problem's stream; returns after the kernel has finished.  Requires hho_setup.
 * Errors: HHO_E_INVALID_ARG (NULL pointer, no setup), HHO_E_LOCAL_SINGULAR. */
int hho_recover_cells(hho_problem *p, const double *x_dev, double *cell_u_dev, double *cell_p_dev);

/* ---- inspection and kernel-level entry points (parity tests, benchmarks) ---- */

/* Condensed right-hand side of level 0 (device, [level-0 size]). */
int hho_get_rhs(hho_problem *p, double *b_dev);

/* Condensed local system of one cell, host buffers, in the cell's local order
 * [faces of T (mesh order) x component x mode ; pressure modes of T]:
 * S [n x n], rhs [n], n = d*card(F_T)*n_F + n_P (level 0).  *n_out receives n;
 * HHO_E_CAPACITY if cap < n*n. */
int hho_get_condensed_cell(hho_problem *p, int64_t cell, double *S, double *rhs, int64_t cap,
                           int64_t *n_out);

/* Host copies of the local HHO operators of one cell before condensation:
 * a [nloc x nloc] scalar viscous matrix (cell modes first, then faces in mesh
 * order), B [d x n_T x nloc], rhs_u [d x nloc], rhs_p [n_T].  With the device
 * build (options.local_build) the records exist after hho_setup, which this
 * call then needs. */
int hho_get_local_cell(const hho_problem *p, int64_t cell, double *a, double *B, double *rhs_u,
                       double *rhs_p, int64_t cap, int64_t *nloc_out);

/* The local operators of the HHO scheme with hybrid pressure (Section 2.3.2,
 * Scheme 2), on the host, for one cell of a mesh: velocity with cell modes of
 * degree k + 1 and face modes of degree k, pressure with cell and face modes of
 * degree k (hierarchical orthonormal bases).  a [nloc x nloc] scalar viscous
 * matrix (the N1 = dim P^{k+1}(T) cell modes first, then the faces in mesh
 * order, dim P^k(F) each), B [d x npl x nloc] pressure-velocity coupling per
 * velocity component (pressure rows: dim P^k(T) cell modes, then dim P^k(F) per
 * face), rhs_u [d x nloc], rhs_p [npl]; nloc = N1 + card(F_T) dim P^k(F),
 * npl = dim P^k(T) + card(F_T) dim P^k(F).  The coupling is used for both the
 * momentum and the mass balance (a symmetric system; the mass datum is
 * (g_D . n_TF, q_F)_F on Dirichlet faces).  eta: Nitsche penalty; qdeg:
 * quadrature degree of the data integrals (>= 2k + 2).  Builds every cell of
 * the mesh (host threads) and copies one; caller-owned host buffers, any of
 * them may be NULL; HHO_E_CAPACITY if cap < max(nloc^2, d npl nloc), the sizes
 * still written.  No device is used. */
int hho_local_hp_cell(const hho_mesh *m, int k, double eta, int qdeg, int64_t cell, hho_field_fn f,
                      hho_field_fn gD, hho_field_fn gN, void *ctx, double *a, double *B, double *rhs_u,
                      double *rhs_p, int64_t cap, int64_t *nloc_out, int64_t *npl_out);

/* The v&p-cond skeleton of the HHO-hp scheme (Section 2.3.2 condensed as in
 * Section 4.1.2), on the host: every cell's velocity and pressure unknowns
 * eliminated (through the Cholesky factor of a_TT and the SPD pressure Schur
 * complement), leaving per face its d velocity components and its pressure,
 * dim P^k(F) modes each; unknown (f (d + 1) + c) dim P^k(F) + j (c = d: the
 * pressure).  CSR in caller-owned host buffers: rowptr [n + 1], col and val
 * [nnz] (rows sorted; every block of a pair of faces of a common cell stored in
 * full), rhs [n].  With a pure Dirichlet boundary the constant face pressure
 * spans the kernel.  Arguments as hho_local_hp_cell; HHO_E_CAPACITY (sizes
 * still written) if cap_nnz < nnz.  No device is used. */
int hho_hp_skeleton(const hho_mesh *m, int k, double eta, int qdeg, hho_field_fn f, hho_field_fn gD,
                    hho_field_fn gN, void *ctx, int64_t *rowptr, int64_t *col, double *val, double *rhs,
                    int64_t cap_nnz, int64_t *n_out, int64_t *nnz_out);

/* y = S_l x on level l in FP64 (device vectors in the global layout). */
int hho_level_apply(hho_problem *p, int level, const double *x_dev, double *y_dev);

/* The level-l operator (which = 0: y = S_l x) or smoother preconditioner
 * (which = 1: y = M_l x) in the V-cycle's own precision: on levels above the
 * coarsest of an HHO_PREC_FP32/BF16 problem, x is rounded to FP32, the stored
 * FP32/bfloat16 values are applied in FP32 arithmetic and y is widened back to
 * FP64; otherwise as hho_level_apply / hho_precond_apply (device vectors). */
int hho_vcycle_level_apply(hho_problem *p, int level, int which, const double *x_dev, double *y_dev);

/* z = M_l r: the level-l smoother preconditioner (cell-patch Schwarz), FP64. */
int hho_precond_apply(hho_problem *p, int level, const double *r_dev, double *z_dev);

/* z = block-triangular preconditioner of the coarsest level applied to v
 * (device vectors of the coarsest level's size, FP64): pressure
 * y_T = -v_T / S_T with S_T = sum_{(f,c) in T} C[(f,c),T]^2 / S[(f,c),(f,c)], velocity
 * one smoothed-aggregation V-cycle on v_f - C y per component.  Only when the
 * problem uses HHO_COARSE_AMG (explicitly or through AUTO). */
int hho_coarse_prec_apply(hho_problem *p, const double *v, double *z);

/* x = the coarsest level's solver applied to b (device vectors of the
 * coarsest level's size, FP64), as inside the V-cycle: the bordered dense
 * inverse, the sparse direct solve (x orthogonal to the constant-pressure null
 * vector when there is one, b first made so), or GMRES to coarse_rtol. */
int hho_coarse_solve_apply(hho_problem *p, const double *b, double *x);

/* The sparse direct solver's symbolic phase (host arrays, as int64), after
 * hho_problem_set_data with HHO_COARSE_DIRECT: "m", "nfs" (unknowns of each front
 * and how many it eliminates), "child" (2 per front, -1 if none), "dofoff",
 * "dof" (the unknowns of each front: its own first, then its update part in
 * elimination order), "cmap" (2 per front position: position in child 0/1's
 * update part, -1 if absent), "hptr"/"hfront" (fronts by tree height), "pinned"
 * (per member of a batch, one for a single problem: the unknown fixed to zero,
 * or -1 when there is no pressure null space), "sizes" (fronts, heights, front entries,
 * factor entries used by the solves, largest front), "hfwd"/"hbwd" (per tree
 * height, two values: the front entries the forward / backward pass reads, and
 * the unknowns of its fronts).  cap: room in out;
 * *n_out receives the length (HHO_E_CAPACITY when it exceeds cap). */
int hho_direct_info(const hho_problem *p, const char *name, int64_t *out, int64_t cap, int64_t *n_out);

/* Host copy of an internal device array for inspection: name "amg_val",
 * "amg_pval", "amg_dinv", "amg_lam", "amg_ainv" (AMG level `level`) or "sd"
 * (pressure Schur approximation).  *n_out receives the length. */
int hho_debug_copy(hho_problem *p, const char *name, int level, double *out, int64_t cap, int64_t *n_out);

/* x = MG_V(0, b, 0): one V-cycle from a zero initial guess, in the problem's
 * V-cycle precision (device vectors, FP64, global layout). */
int hho_vcycle_apply(hho_problem *p, const double *b_dev, double *x_dev);

/* Average duration in ms of `reps` back-to-back launches, bracketed by HIP
 * events on the problem's stream, of one kernel on level `level`:
 * kind 0 = FP64 operator application y = S_l x, 1 = FP64 Schwarz preconditioner,
 * 2 = the V-cycle's operator application (two-slot input, V-cycle precision),
 * 3 = one full V-cycle from level 0.  Inputs are fixed internal vectors. */
int hho_time_kernel(hho_problem *p, int kind, int level, int reps, double *avg_ms);

/* Autotuner: times candidate launch shapes on the problem's own data (reps
 * launches each) and keeps the fastest per level: threads per block of the
 * operator kernels (64, 128, 256) and threads per cell of the smoother patch
 * factorisation (64, 128, 256, 512).  choices (may be NULL) receives 2 ints per
 * level (operator block, patch threads; 0 = level without a smoother).  The
 * factorisations are recomputed while timing, so hho_setup must be called again
 * before hho_solve. */
int hho_autotune(hho_problem *p, int reps, int *choices);

/* Phase timings of the last hho_setup / hho_solve in milliseconds (device
 * events): [0] condensation, [1] assembly, [2] levels, [3] smoother setup,
 * [4] coarse setup, [5] solve, [6] V-cycle total, [7] V-cycle count,
 * [8] coarse iterations total.  n is the capacity of t. */
int hho_get_timings(const hho_problem *p, double *t, int n);

/* ---- live kernel timing (measurement) ----
 * Classes of kernel launches that hho_solve can time while it runs: each armed
 * launch is bracketed by two HIP events recorded on the problem's stream (the
 * stream the kernel runs on), and hho_probe_read sums the elapsed times.  The
 * events add a few microseconds of ordering between launches; disarm (mask 0)
 * for untimed runs.  "level" is the V-cycle level for the first three classes,
 * the level of the coarse preconditioner's aggregation hierarchy for the AMG
 * classes (Section 5.2's iterative coarsest-level solve, preconditioned). */
#define HHO_PROBE_OPERATOR         1   /* operator application of a smoothing step (Section 3.3), level l */
#define HHO_PROBE_SMOOTHER         2   /* cell-patch Schwarz preconditioner of a smoothing step, level l   */
#define HHO_PROBE_COARSE_OPERATOR  4   /* coarsest-level operator inside the coarse GMRES                  */
#define HHO_PROBE_OUTER_OPERATOR   8   /* FP64 level-0 operator of each FGMRES iteration                   */
#define HHO_PROBE_AMG_RESTRICT    16   /* AMG restriction of the pre-smoothed residual, AMG level l         */
#define HHO_PROBE_AMG_SWEEP       32   /* AMG damped-Jacobi sweeps, AMG level l                             */
#define HHO_PROBE_AMG_PROLONG     64   /* AMG prolongation with the first post-sweep, AMG level l           */
#define HHO_PROBE_AMG_DENSE      128   /* AMG explicit small-level operator or dense coarsest inverse       */
#define HHO_PROBE_DIRECT_FWD     256   /* sparse direct coarse solve, forward pass, tree height l           */
#define HHO_PROBE_DIRECT_BWD     512   /* sparse direct coarse solve, backward pass, tree height l          */
#define HHO_PROBE_ALL           1023

/* Arms the classes of `mask` (0 disarms) and discards recorded launches; every
 * stride-th launch (>= 1) of each armed class and level is timed, the first one
 * included, so that the event calls do not hold up a stream of short launches. */
int hho_probe_arm(hho_problem *p, unsigned mask, int stride);
/* Timed launches of class `kind` (one HHO_PROBE_* bit) on `level` (-1: every
 * level) and their summed duration in ms, since the last arm/clear; launches
 * (may be NULL) receives every launch of that class and level, timed or not.
 * Synchronises the problem's stream.  HHO_E_DEVICE if an event failed. */
int hho_probe_read(hho_problem *p, int kind, int level, int64_t *timed, double *total_ms, int64_t *launches);
/* Discards recorded launches (the armed classes stay armed). */
int hho_probe_clear(hho_problem *p);
/* Sizes of level `level` of the coarse preconditioner's aggregation hierarchy
 * (problems whose coarsest solver is HHO_COARSE_AMG, after hho_problem_set_data):
 * info[0] rows n, [1] coarse rows of the next level (0 on the last), [2] entries
 * of A, [3] of the prolongator P, [4] of B = A P, [5] the first level applied as
 * an explicit matrix (-1: none; set by the workspace plan), [6] number of levels. */
int hho_amg_level_info(const hho_problem *p, int level, int64_t *info);

/* ---- batches of independent problems (not in the paper) ----
 * n meshes become one mesh (their disjoint union; member i's faces and cells
 * keep their order and follow those of members 0..i-1), a problem on it is told
 * the member ranges with hho_problem_set_segments, and hho_solve then runs one
 * flexible GMRES process per member: the V-cycle and the operator act on the
 * whole union at once (block diagonal), while the Arnoldi dot products,
 * Hessenberg columns, Givens rotations, restarts and the stopping test
 * (true relative residual of each member <= rtol) are per member.  Members with
 * a pure Dirichlet boundary have their own constant-pressure null vector. */

/* Disjoint union of n meshes (host descriptors, copied).  face_offsets and
 * cell_offsets (may be NULL, else n+1 entries) receive the first face / cell
 * of every member and the totals. */
int hho_mesh_create_union(const hho_mesh_desc *descs, int n, hho_mesh **out, int64_t *face_offsets,
                          int64_t *cell_offsets);

/* Declares the members of a union mesh: member i owns faces [face_ptr[i],
 * face_ptr[i+1]) and cells [cell_ptr[i], cell_ptr[i+1]) (partitions, every
 * cell's faces in its own member).  Call after hho_problem_create and before
 * hho_problem_set_data.  Each member is the problem it would be alone: with the
 * default penalty (options.eta <= 0) its cells take 4(k+1)(k+d)/d times the
 * member's own max card(F_T).  Either every member or none may have Neumann
 * faces (HHO_E_INVALID_ARG otherwise): a pure-Dirichlet member has its own
 * constant-pressure null vector.  A dense coarsest-level solver is refused when
 * the members have a pressure null space (use AMG or GMRES). */
int hho_problem_set_segments(hho_problem *p, int n, const int64_t *face_ptr, const int64_t *cell_ptr);

/* After a batched hho_solve: FGMRES iterations and final true relative
 * residual of every member (host arrays of n = number of members). */
int hho_batch_results(const hho_problem *p, int *iters, double *rel, int n);

/* Batches built from separately created problems (the same combined problem as
 * above, assembled by the library): n problems with equal dimension, degree
 * schedule, condensation variant and solver options (the penalty eta may
 * differ), each after hho_problem_set_data.  The batch copies the meshes and
 * local operators (members may be destroyed afterwards) and owns one combined
 * problem, returned by hho_batch_problem: query its workspace size, bind a
 * workspace and stream, and call hho_setup on it as on any problem. */
typedef struct hho_batch hho_batch;
int hho_batch_create(hho_problem *const *ps, int n, hho_batch **out);
void hho_batch_destroy(hho_batch *b);
int hho_batch_problem(hho_batch *b, hho_problem **p);
/* face_n[i], p_n[i]: hho_solve's output sizes of member i (host arrays of n). */
int hho_batch_sizes(const hho_batch *b, int64_t *face_n, int64_t *p_n);
/* Solves every member (one flexible GMRES process each, one V-cycle over the
 * union).  Member i's face modes go to face_out[face_off[i] .. face_off[i+1]),
 * its cell pressure modes to p_out[p_off[i] .. p_off[i+1]) (host, layouts as in
 * hho_solve; ranges at least hho_batch_sizes long, else HHO_E_CAPACITY before
 * any work).  Host arrays of n (may be NULL): iters, final_rel (true relative
 * residual), status (HHO_OK or HHO_E_NOT_CONVERGED); hist with hist_off (n+1
 * entries; may be NULL) receives member i's relative residual estimates, entry 0
 * = 1, one per Arnoldi step it took, truncated to its range.  Returns HHO_OK
 * when every member converged, else HHO_E_NOT_CONVERGED. */
int hho_batch_solve(hho_batch *b, double *face_out, const int64_t *face_off, double *p_out, const int64_t *p_off,
                    int *iters, double *hist, const int64_t *hist_off, double *final_rel, int *status);

/* ---- learned fine-level smoother (not in the paper) ----
 * Needs a problem created with options.learned = 1 and a bound workspace.
 * Per face F of level 0 a network maps a window of the residual r to a
 * correction of F's d*n_F velocity unknowns and of the n_P pressure unknowns of
 * each of F's cells:
 *   window: for the cells T_0 < T_1 of F (T_1 absent on the boundary), the
 *     residual blocks of T_s's faces in its face order, zero padded to Fm (the
 *     largest card(F_T) of the mesh), then T_s's pressure residual; then one-hots
 *     of F's position in T_0's and T_1's face lists:
 *     n_in = 2 (Fm d n_F + n_P) + 2 Fm entries;
 *   scale s_F = root mean square of the residual part (over 2 (Fm d n_F + n_P)
 *     entries), which is divided by s_F;
 *   h = relu(W1 x + b1) (64 units), y = W2 h + b2 (n_out = d n_F + 2 n_P);
 *   correction: s_F y[0 .. d n_F) on F's velocity unknowns; each cell T takes
 *     the mean over its faces F of s_F y[d n_F + side n_P ..] (side = T's
 *     position in F's cell pair) on its pressure unknowns.
 * The products run on bfloat16 x, W1, h and W2 (rounded to nearest even) with
 * FP32 sums on the matrix cores; biases, outputs and the master parameters are
 * FP32: [W1 (64 x n_in, row-major) | b1 | W2 (n_out x 64) | b2].  Gradients are
 * those of this network with the roundings taken as the identity.
 * When enabled, every level-0 smoothing step minimises the residual over the
 * Schwarz directions plus this correction, so its residual never exceeds the
 * plain step's: the plain smoother is both the fallback and the yardstick. */

/* Sizes of the network: inputs, outputs, hidden units and parameter count. */
int hho_learned_dims(const hho_problem *p, int *n_in, int *n_out, int *hidden, int64_t *n_params);

/* Copy parameters in (host, exactly n_params floats); resets the Adam moments. */
int hho_learned_set_params(hho_problem *p, const float *params, int64_t n);

/* Copy the current parameters out (host, exactly n_params floats). */
int hho_learned_get_params(const hho_problem *p, float *params, int64_t n);

/* Parameters as bytes: a 32-byte header (magic "HHOMLP01", int32 n_in, n_out,
 * hidden, 0, int64 n_params) followed by the n_params FP32 values in the layout
 * above, host byte order.  hho_learned_save writes them to buf (host, cap
 * bytes; *need receives the size, buf may be NULL to query it: HHO_E_CAPACITY);
 * hho_learned_load reads them back (HHO_E_INVALID_ARG when the sizes differ
 * from the problem's network) and resets the Adam moments. */
int hho_learned_save(const hho_problem *p, void *buf, size_t cap, size_t *need);
int hho_learned_load(hho_problem *p, const void *buf, size_t n);

/* Use (on = 1) or stop using (0) the learned direction in level-0 smoothing. */
int hho_learned_enable(hho_problem *p, int on);

/* z = correction of every face for the level-0 residual r (device, FP64 in and
 * out, network in FP32); cell entries of z are 0.  Needs hho_setup. */
int hho_learned_apply(hho_problem *p, const double *r_dev, double *z_dev);

/* Training pairs from the plain V-cycle: with b = S_0 x_true and x = 0, for
 * each of `cycles` iterations the windows of r = b - S_0 x and the targets
 * ((x_true - x) on F, on T_0, on T_1) / s_F of every face (0 for an absent T_1)
 * are written (rows cycle*n_faces + F of X [cap x n_in] and T [cap x n_out],
 * device FP32), then x += MG_V(r).
 * *n_out = cycles * n_faces; HHO_E_CAPACITY if cap is smaller. */
int hho_learned_collect(hho_problem *p, const double *x_true_dev, int cycles, float *X_dev, float *T_dev,
                        int64_t cap, int64_t *n_out);

/* Loss 1/(2n) sum_i |y(X_i) - T_i|^2 and its gradient (host, n_params floats,
 * same layout as the parameters) over the n rows of X, T (device, 1 <= n <= 4096). */
int hho_learned_grad(hho_problem *p, const float *X_dev, const float *T_dev, int64_t n, float *grad,
                     double *loss);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): the same loss and gradient
 * as hho_learned_grad, with the same kernels in the same order (so the results
 * are identical), but the work arrays -- hidden activations and outputs of the
 * batch and their gradients, the parameter gradient, the loss partial sums --
 * live in a fixed device array of the library (about 14 MiB per device, held
 * until the process ends) instead of the problem's workspace.  The call itself
 * allocates nothing.  Limits: 1 <= n <= 4096 rows, n_out <= 256 outputs,
 * n_params <= 2^20; beyond them it returns HHO_E_CAPACITY.  The device of the
 * problem's workspace must be current (HHO_E_INVALID_ARG otherwise).  Every
 * call on one device shares that array: calls that overlap on one device (other
 * host threads, other streams) race and must be serialised by the caller. */
int hho_learned_grad_noalloc(hho_problem *p, const float *X_dev, const float *T_dev, int64_t n, float *grad,
                             double *loss);

/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on
 * batches of `batch` rows (<= 4096) drawn from the n rows of X, T: row i of the
 * batch of step s (counted from 0 since the last hho_learned_set_params, across
 * calls) is SM(seed ^ SM((s << 32) | i)) mod n, SM the SplitMix64 output
 * function (Steele, Lea & Flood 2014); loss_hist (host, may be NULL) receives the
 * batch loss of every step. */
int hho_learned_train(hho_problem *p, const float *X_dev, const float *T_dev, int64_t n, int steps, int batch,
                      float lr, uint64_t seed, float *loss_hist);

#ifdef __cplusplus
}
#endif
#endif /* HHO_PMG_H */
