/*
 * seird.h -- C ABI of libseird: the backward-Euler implicit step of the
 * five-compartment SEIRD reaction-diffusion model on P1 triangles, solved by
 * Newton's method with GMRES preconditioned by restricted additive Schwarz
 * (one-level, or multiplicative two-grid with a nested coarse grid), on
 * AMD Instinct MI355X (gfx950).
 *
 * The model is the PDE system of Section 2.1 (Eqs. seird1-seird5, N):
 *   d_t u - div(nu(u) grad u) = B(u) u,   u = (s, e, i, r, d),
 *   nu(u) = N diag(nu_S, nu_E, nu_I, nu_R, nu_D)      (Eq. vec_component1)
 *   B(u) the reaction matrix of Eq. vec_component2,
 * discretised by backward Euler (Eq. timediscrete) and the weak form
 * (Eq. weakform) on P1 triangles, homogeneous Neumann data and lumped nodal
 * mass by default (see seird_set_mass and seird_set_boundary_flux for the
 * variants), nodal quadrature of the reaction, exact P1 diffusion with the
 * element-mean density.  The discrete residual of one step is
 *
 *   F_{c,i}(u) = m_i (u_{c,i} - u^n_{c,i})
 *              + dt nu_c sum_{T ni i} Nbar_T sum_{j in T} K^T_{ij} u_{c,j}
 *              - dt m_i R_c(u_i) - dt m_i src_{c,i}
 *
 * with m_i the lumped mass, K^T_{ij} = |T| grad(phi_i).grad(phi_j),
 * Nbar_T the mean of N over the vertices of T and R_c the nodal reaction
 * (B(u)u)_c.  An optional per-node transmission field g multiplies beta_I
 * and beta_E (the product form of Eq. beta_ie).
 *
 * Conventions for every call:
 *  - State and vectors are device pointers to contiguous float64 arrays in
 *    node-major layout [n_nodes][5] (unknown 5*node + c, c = S,E,I,R,D),
 *    owned by the caller and only borrowed for the duration of the call.
 *  - Mesh and partition arrays are host pointers; they are copied.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Calls that only launch work are asynchronous on that stream;
 *    calls documented as synchronising wait for it before returning.
 *  - Every call returns a seird_status; on failure seird_last_error()
 *    returns a message (thread-local).  No exception crosses the ABI.
 *  - Handles are not thread-safe; calls on one handle must not overlap.
 *  - The library allocates its own device memory at create time (freed by
 *    the matching destroy), unless the problem was created inside a
 *    caller-owned workspace (seird_create_in_workspace).
 */
#ifndef SEIRD_H
#define SEIRD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int seird_status;
#define SEIRD_OK 0
#define SEIRD_ERR_ARG (-1)           /* invalid argument or size */
#define SEIRD_ERR_MESH (-2)          /* degenerate or invalid mesh */
#define SEIRD_ERR_HIP (-3)           /* HIP runtime error (sticky) */
#define SEIRD_ERR_NONFINITE (-4)     /* NaN/Inf in a state or residual */
#define SEIRD_ERR_BREAKDOWN (-5)     /* zero or tiny pivot in a local LU */
#define SEIRD_ERR_DIVERGED (-6)      /* GMRES residual > dtol * ||b|| */
#define SEIRD_ERR_NOT_CONVERGED (-7) /* iteration cap reached */
#define SEIRD_ERR_WORKSPACE (-8)     /* caller workspace too small or not reserved for this use */
#define SEIRD_ERR_STATE (-9)         /* total density N <= 0 at a node */

typedef struct seird_problem_s *seird_problem;
typedef struct seird_precond_s *seird_precond;

/* Model parameters (Section 2.1, Table 1).  Rates per unit time, A in
 * density units, beta_I/beta_E per density unit per time, nu[c] in
 * length^2 per density unit per time.  alpha, mu: vital dynamics. */
typedef struct {
  double sigma, gamma_E, gamma_R, gamma_D, A, alpha, mu, beta_I, beta_E;
  double nu[5];
} seird_params;

/* Schwarz preconditioner options (Section 3).
 *  n_sub, part: node partition into owner subdomains (part[node] in
 *    [0, n_sub)); subdomain i is its owner set grown by `overlap` layers of
 *    mesh-graph neighbours; D_i is the Boolean owner indicator (Eq. RAS).
 *  tile: tile edge of the local factors' storage (16 or 32).  Each
 *    subdomain's factors are kept in its tile envelope: tile row K stores
 *    the tiles from its first nonzero tile column (nondecreasing down the
 *    rows, so that LU without pivoting fills only inside) to the symmetric
 *    upper extent.
 *  factor_prec: storage precision of the local factors used by the
 *    preconditioner apply: 0 = float64, 1 = float32, 2 = bfloat16.  With
 *    tile 32 and factor_prec 1 or 2 the subdomain factorisation runs in
 *    float32 on the float32 MFMA (float32 accumulation); factor_prec 2 then
 *    rounds the float32 factors to bfloat16 for the apply (each tile as it
 *    becomes final).  With tile 16
 *    the factorisation runs in float64 and the factors are rounded to the
 *    storage precision.  The coarse factorisation is always float64, and
 *    the vectors and accumulations of the apply stay float64.
 *  Two-grid (multiplicative, Eqs. presmoother/coarsecorrection/
 *  postsmoother): n_ref > 0 enables it.  The coarse grid is nested: level 0
 *  has level_n[0] nodes and refinement record r (1..n_ref) maps each of
 *  the level_n[r] nodes of level r to the two level-(r-1) nodes whose edge
 *  it bisects ((p, p) for a node carried over), parents[] holding the
 *  records back to back as int32 pairs; level_n[n_ref] must equal n_nodes
 *  and follow the problem's node numbering.  Z is the P1 interpolation
 *  from level 0; the coarse matrix is the Galerkin product Z^T A Z,
 *  factored exactly in float64. */
typedef struct {
  int32_t n_sub;
  int32_t overlap;
  int32_t tile;
  int32_t factor_prec;
  int32_t n_ref;
  const int64_t *level_n;  /* host, n_ref + 1 entries, or NULL */
  const int32_t *parents;  /* host, sum_{r>=1} 2*level_n[r] entries */
} seird_schwarz_opts;

/* GMRES options (Section 3.2): right preconditioning, x0 = 0, restart
 * length, total iteration cap, convergence ||r|| < max(rtol ||b||, atol),
 * divergence ||r|| > dtol ||b||.  Classical Gram-Schmidt with one
 * conditional reorthogonalisation pass.
 * graphs = 1: the launches of every Arnoldi step (preconditioner apply,
 * SpMV, projections) are captured once per basis index into a HIP graph,
 * cached on the preconditioner, and replayed; results are identical to
 * direct launches (graphs = 0).  Ignored while preconditioner timing is on
 * or without a preconditioner. */
typedef struct {
  int32_t restart;
  int32_t max_it;
  double rtol, atol, dtol;
  int32_t graphs;
} seird_krylov_opts;

typedef struct {
  int32_t its;
  int32_t reason; /* 1 rtol/atol, 2 happy breakdown, -6 diverged, -7 max_it */
  double resid;   /* final residual estimate */
  double bnorm;
} seird_krylov_stats;

/* Newton options: stop when ||F(u^k)||_2 <= tol * ||M_L u^n||_2, at most
 * max_it linear solves.  pc_reuse: a preconditioner setup serves this many
 * further Newton iterations of the same step before it is rebuilt (0 = a
 * fresh setup at every iteration; the converged root does not depend on
 * it, only the GMRES iteration counts do).  strict_linear: when GMRES stops
 * at its max_it without reaching its tolerance inside a Newton iteration,
 * 1 fails the step with SEIRD_ERR_NOT_CONVERGED; 0 takes the inexact
 * update (inexact Newton) and counts it in seird_step_stats.inexact_solves.
 * pc_keep_steps: a setup made by a step may also serve the first
 * iterations of this many later steps of the same problem and dt (0 = a
 * fresh setup at every step's first iteration); a kept setup whose GMRES
 * fails or needs more than twice its fresh count plus 5 is rebuilt, as a
 * reused one within a step.  A setup made outside the step calls is never
 * kept.  In seird_forward_record the kept setups restart at every
 * checkpoint (so that seird_adjoint's recomputation of a segment repeats
 * its steps exactly), and seird_adjoint's transposed solves keep their
 * setups for as many further reverse steps of a segment. */
typedef struct {
  double tol;
  int32_t max_it;
  int32_t pc_reuse;
  int32_t strict_linear;
  int32_t pc_keep_steps;
} seird_newton_opts;

#define SEIRD_MAX_NEWTON 32
typedef struct {
  int32_t newton_its;
  int32_t gmres_its_total;
  int32_t gmres_its[SEIRD_MAX_NEWTON];
  double res_hist[SEIRD_MAX_NEWTON + 1]; /* scaled residuals */
  double eps;      /* ||u^{k+1}-u^k|| / ||u^n|| of the last update (Eq. picardtol) */
  int32_t reason;  /* SEIRD_OK or the failing status */
  int32_t pc_setups; /* preconditioner setups done in this step */
  double t_residual_ms, t_jacobian_ms, t_setup_ms, t_gmres_ms;
  /* HIP-event time of the subdomain solve launches (the RAS apply kernel)
   * during this step, their count, and the bytes a launch reads/writes by
   * the algorithm (factor storage + local vectors), averaged over the
   * launches (in a batch, subdomains of converged instances are skipped
   * and not counted). */
  double t_ras_kernel_ms;
  int32_t n_ras_launches;
  double ras_bytes_per_launch;
  /* halvings of Newton updates in this step: an update after which the
   * total density N is <= 0 at some node is halved (at most 10 times per
   * update, else SEIRD_ERR_STATE) */
  int32_t backtracks;
  /* Newton iterations of this step whose GMRES stopped at max_it without
   * reaching its tolerance (their inexact updates were taken) */
  int32_t inexact_solves;
} seird_step_stats;

/* ------------------------------------------------------------------
 * Meshes and caller-owned workspaces.
 * A mesh handle holds host data only (node graph, element incidence,
 * lumped mass); problems are created from it either with library-owned
 * device memory (seird_problem_create_from_mesh) or inside one device
 * workspace the caller allocated (seird_create_in_workspace), in which
 * case the library calls no hipMalloc for the problem, its preconditioner,
 * their solves, steps and adjoint records.
 * ------------------------------------------------------------------ */
typedef struct seird_mesh_s *seird_mesh;
/* What a workspace reserves beyond the problem and its preconditioner:
 *  restart_max: the largest GMRES restart any solve will use (the Krylov
 *    basis V [restart_max + 1][N] and Z [restart_max][N] are reserved;
 *    a larger restart later fails with SEIRD_ERR_WORKSPACE);
 *  tape_states: state vectors [n][5] for adjoint records: a record of
 *    n_steps with checkpoints every c steps needs ceil(n_steps / c) + c + 4
 *    (checkpoints, one segment's states, the adjoint vectors); 0 = no
 *    adjoint records (seird_forward_record then fails with
 *    SEIRD_ERR_WORKSPACE);
 *  n_regions_max: the most observation regions of a record;
 *  csr_pattern: 1 keeps room for seird_csr's pattern (25 (n_slots + n)
 *    int32 columns and 5 n + 1 int64 row offsets). */
typedef struct {
  int32_t restart_max;
  int32_t tape_states;
  int32_t n_regions_max;
  int32_t csr_pattern;  /* 1: keep room for the scalar CSR pattern of seird_csr */
} seird_workspace_opts;

/* Validate and build a triangle mesh (host arrays copied; no device
 * memory).  Errors as seird_problem_create. */
seird_status seird_mesh_create(int64_t n_nodes, const double *xy, int64_t n_tri,
                               const int32_t *tri, seird_mesh *out);
void seird_mesh_destroy(seird_mesh m);
seird_status seird_mesh_info(seird_mesh m, int64_t *n_nodes, int64_t *n_slots);
/* A problem on the mesh with library-owned device memory (the mesh data are
 * copied; the mesh may be destroyed afterwards). */
seird_status seird_problem_create_from_mesh(seird_mesh m, const seird_params *params,
                                            seird_problem *out);
/* Bytes of device workspace that seird_create_in_workspace needs for this
 * mesh, preconditioner (opts and part as seird_precond_create; opts = NULL:
 * no preconditioner) and reservation.  Host only: no device call. */
seird_status seird_workspace_bytes(seird_mesh m, const seird_schwarz_opts *opts,
                                   const int32_t *part, const seird_workspace_opts *wo,
                                   int64_t *bytes);
/* Create the problem (and, with opts, its preconditioner) with every device
 * array inside ws (device memory of ws_bytes bytes, 256-byte aligned, owned
 * by the caller, which keeps it allocated until both handles are
 * destroyed; destroy the preconditioner before the problem).
 * SEIRD_ERR_WORKSPACE if ws_bytes is below seird_workspace_bytes.  The
 * handles are used as any others; what allocates nothing here: the setup,
 * apply, SpMV, assembly, GMRES (restart <= restart_max, graphs = 0),
 * step, forward record and adjoint calls (HIP graphs, which the runtime
 * allocates for, stay available with graphs = 1). */
seird_status seird_create_in_workspace(seird_mesh m, const seird_params *params,
                                       const seird_schwarz_opts *opts,
                                       const int32_t *part,
                                       const seird_workspace_opts *wo, void *ws,
                                       int64_t ws_bytes, seird_problem *prob,
                                       seird_precond *pc);

const char *seird_last_error(void);
/* Device allocations (hipMalloc calls) the library has made in this
 * process, and their bytes: lets a caller check that calls on workspace
 * handles allocate nothing. */
seird_status seird_device_allocations(int64_t *count, int64_t *bytes);
/* Version string of the library (build identifier). */
const char *seird_version(void);

/* Create a problem on the current HIP device from a triangle mesh.
 *  xy: host float64 [n_nodes][2]; tri: host int32 [n_tri][3] (either
 *  orientation).  Returns SEIRD_ERR_MESH for out-of-range indices, repeated
 *  vertices or zero-area triangles.  Builds the node graph, the element
 *  incidence records and the lumped mass (Section 2.2). */
seird_status seird_problem_create(int64_t n_nodes, const double *xy,
                                  int64_t n_tri, const int32_t *tri,
                                  const seird_params *params,
                                  seird_problem *out);
void seird_problem_destroy(seird_problem p);
seird_status seird_set_params(seird_problem p, const seird_params *params);
/* ------------------------------------------------------------------
 * Model and discretisation variants (Section 4.2, Appendix B.3).
 * ------------------------------------------------------------------
 * Time profile of the transmission rate (Eq. beta_ie): with a schedule,
 * beta_I and beta_E are multiplied by a - b / (1 + exp(k (tc - t))) at the
 * time t the coefficients refer to: the end of a step (t_n + dt) in
 * seird_step, seird_pgs_step and the forward/adjoint sweeps, the problem's
 * time in seird_residual and seird_jacobian.  NULL removes it.  The paper's
 * profile is a = 0.101, b = 0.05, k = 1 per day, tc = 130 days.  Not for a
 * batch's problem (SEIRD_ERR_ARG). */
typedef struct {
  double a, b, k, tc;
} seird_beta_schedule;
seird_status seird_set_beta_schedule(seird_problem p, const seird_beta_schedule *s);
/* Model time of the current state: set by the caller, advanced by dt by
 * every successful step (and by n_steps dt by a forward record). */
seird_status seird_set_time(seird_problem p, double t);
seird_status seird_get_time(seird_problem p, double *t);
/* Regional transmission profile along the first coordinate (Eq. beta_x):
 * sets the transmission field to
 *   g(x) = beta_c + (beta_e - beta_c) / (1 + exp(-k_e (x - x_e)))
 *               + (beta_w - beta_c) / (1 + exp(k_w (x - x_w)))
 * at every node (the paper's k_e = 5, k_w = 10).  Synchronising. */
seird_status seird_set_beta_regional(seird_problem p, double beta_c, double beta_e,
                                     double beta_w, double x_e, double x_w,
                                     double k_e, double k_w, void *stream);
/* Mass of the time-derivative term: 0 lumped (default), 1 consistent
 * (M_ij = int phi_i phi_j, so the term is sum_j M_ij (u - u^n)_j; the
 * reaction keeps nodal quadrature and the Newton stopping scale stays
 * ||M_L u^n||).  The Jacobian, preconditioners, Picard-Gauss-Seidel sweeps
 * and the adjoint follow. */
seird_status seird_set_mass(seird_problem p, int32_t consistent);
/* Non-homogeneous Neumann data: the flux vector field q = nu(u) grad u of
 * every compartment at every node, device float64 [n_nodes][5][2]
 * (copied; only boundary nodes matter).  The residual then subtracts
 * dt int_{boundary} (q . n) phi_i ds, with q P1 along each boundary edge
 * and n the edge's outward normal (Eq. weakform's boundary term, taken as
 * data that does not depend on the state).  NULL restores homogeneous
 * Neumann.  Async. */
seird_status seird_set_boundary_flux(seird_problem p, const double *q_dev, void *stream);

/* Per-node transmission multiplier g [n_nodes] (device float64, copied);
 * NULL restores g = 1. */
seird_status seird_set_beta_field(seird_problem p, const double *g_dev,
                                  void *stream);
seird_status seird_problem_info(seird_problem p, int64_t *n_nodes,
                                int64_t *n_slots);
/* Node graph of the Jacobian (host copies): rowptr [n_nodes+1] and
 * col [n_slots] list, for every node, its mesh neighbours (itself
 * excluded) in increasing order.  Either pointer may be NULL. */
seird_status seird_pattern(seird_problem p, int64_t *rowptr, int32_t *col);
/* Lumped mass m_i (device float64 [n_nodes], written). */
seird_status seird_lumped_mass(seird_problem p, double *m_dev, void *stream);

/* F = residual of one backward-Euler step (formula above) at u, given
 * u_prev = u^n.  src: optional nodal forcing [n][5] (NULL = 0).  Async. */
seird_status seird_residual(seird_problem p, const double *u,
                            const double *u_prev, double dt, const double *src,
                            double *F, void *stream);

/* Exact Jacobian dF/du at u (Newton linearisation of the weak form).
 * Storage (device float64, caller-owned, seird_jacobian_size values):
 *   diag [n_nodes][5][5]   : node block (row = equation c, col = unknown c')
 *   off  [n_slots][10]     : for slot (i, j) of the node graph, a[5] then
 *                            b[5]; block (i,j)[c][c'] = a[c] delta_cc' + b[c]
 * (the off-diagonal blocks are diagonal-plus-rank-one because N sums all
 * five compartments).  Async. */
seird_status seird_jacobian_size(seird_problem p, int64_t *n_vals);
seird_status seird_jacobian(seird_problem p, const double *u, double dt,
                            double *vals, void *stream);
/* The Jacobian as a scalar CSR matrix of N = 5 n_nodes rows: row 5 i + c
 * holds, for every node j of {i} and its mesh neighbours in increasing
 * order, the five columns 5 j .. 5 j + 4 (block (i, j) of the node-block
 * storage, row c, including its structural zeros), so nnz = 25 (n_slots +
 * n_nodes).  seird_csr returns the pattern: device int64 rowptr [N + 1]
 * and int32 col [nnz], owned by the problem (built on the first call,
 * read-only, valid until the problem is destroyed); seird_csr_values
 * writes the values of node-block Jacobian `vals` in that order into the
 * caller's device array csr_vals [nnz] (async).  SEIRD_ERR_WORKSPACE for a
 * workspace problem created without csr_pattern. */
seird_status seird_csr(seird_problem p, const int64_t **rowptr, const int32_t **col,
                       int64_t *nnz, int64_t *nrows);
seird_status seird_csr_values(seird_problem p, const double *vals, double *csr_vals,
                              void *stream);
/* y = J x (transpose = 0) or y = J^T x (transpose = 1).  Async. */
seird_status seird_spmv(seird_problem p, const double *vals, const double *x,
                        double *y, int transpose, void *stream);

/* Schwarz preconditioner for this problem. */
seird_status seird_precond_create(seird_problem p,
                                  const seird_schwarz_opts *opts,
                                  const int32_t *part, seird_precond *out);
void seird_precond_destroy(seird_precond pc);
/* Local sizes: for subdomain s, the number of local nodes, the node
 * bandwidth of its local ordering, and the factor storage (entries). */
seird_status seird_precond_info(seird_precond pc, int64_t *factor_entries,
                                int64_t *coarse_n, int32_t *max_local_nodes,
                                int32_t *max_bandwidth);
/* Host-only analysis of the Schwarz decomposition (no device calls):
 * builds the mesh graph, subdomains, local orderings and tile
 * envelopes exactly as seird_precond_create does and reports their sizes.
 * l2g_out [local_unknowns] (nullable) receives, subdomain after
 * subdomain, the global unknown of every local unknown in local order;
 * owned_out [local_unknowns] (nullable) its owner flag (D_i). */
typedef struct {
  int64_t factor_entries;   /* stored tile entries: subdomain envelopes + coarse band */
  int64_t local_unknowns;   /* sum of subdomain sizes (unknowns) */
  int32_t max_local_nodes;
  int32_t max_bandwidth;    /* node bandwidth of the local orderings */
  double mean_bandwidth;
  int64_t coarse_n;
  int32_t coarse_bandwidth;
  /* flops of one subdomain factorisation (see seird_precond_perf) */
  double lu_mfma_flops, lu_useful_flops;
} seird_schwarz_info;
seird_status seird_analyze_schwarz(int64_t n_nodes, const double *xy,
                                   int64_t n_tri, const int32_t *tri,
                                   const seird_schwarz_opts *opts,
                                   const int32_t *part,
                                   seird_schwarz_info *info, int32_t *l2g_out,
                                   uint8_t *owned_out);

/* Enable (1) or disable (0) HIP-event timing of the subdomain solve
 * launches; the totals are reported in seird_step_stats (t_ras_kernel_ms,
 * n_ras_launches) and reset at the end of every seird_step. */
seird_status seird_precond_timing(seird_precond pc, int enable);
/* Work figures of the preconditioner and, while timing is on
 * (seird_precond_timing), HIP-event times of its setups: the extraction of
 * the local matrices and the subdomain factorisation, summed over the
 * setups since the last reset (reset != 0 clears them after reading).
 * lu_mfma_flops: flops of one subdomain factorisation as the matrix cores
 * execute them (every tile product at 2 T^3); lu_useful_flops: the same
 * with the triangular panel products at T^3, plus the diagonal tiles' LU
 * and inverses (4/3 T^3 each).  factor_bytes: bytes of the subdomain
 * factors as factorised; solve_bytes: algorithmic bytes of one subdomain
 * solve launch (factors in the storage precision plus local vectors). */
typedef struct {
  double lu_mfma_flops, lu_useful_flops;
  double factor_bytes, solve_bytes;
  int32_t setups;
  double t_extract_ms, t_lu_ms;
} seird_precond_perf_report;
seird_status seird_precond_perf(seird_precond pc, seird_precond_perf_report *r,
                                int reset);
/* Coarse solver of a two-level preconditioner.  3: the Krylov-AMG coarse
 * solver of seird_precond_set_coarse_amg, 2: the Krylov-RAS coarse solver
 * of seird_precond_set_coarse_krylov (once set).  1: the inverses of the
 * diagonal super-blocks of the coarse factors, X_II = L_II^{-1} and
 * W_II = U_II^{-1}, are formed at every setup (FP64 MFMA, on the coarse
 * stream) and A_c^{-1} r is a block forward/backward sweep: per block a
 * dense triangular mat-vec over the device plus a coupling update from the
 * neighbouring block (see seird_precond_set_coarse_block); the default with
 * tile 32 when the storage fits 16 GB (nt(nt+1) tiles of 8 KB for nt coarse
 * tile rows, whatever the block size).  0: the band forward/backward sweeps
 * over the factors (one workgroup).  Results of 0 and 1 agree to rounding.
 * SEIRD_ERR_ARG for 1 without inverses, 2 or 3 without their Krylov
 * coarse solver. */
seird_status seird_precond_set_coarse_solver(seird_precond pc, int32_t solver);
/* Two-grid RAS-V2 (Section 3.2, compared with the direct coarse solve in
 * Table 2 of Section 4.1): the coarse system A_c x_c = Z^T r is solved by an
 * inner GMRES (x0 = 0, right preconditioning) with one-level RAS on the
 * coarse graph, instead of the coarse factorisation.  A_c is the Galerkin
 * matrix Z^T A Z held as dense 5x5 node blocks of the coarse graph.  Coarse
 * subdomains: each coarse node belongs to the fine subdomain that owns the
 * fine node carrying its largest interpolation weight (its own node on a
 * nested grid), so the coarse problem is split like the fine one; n_sub > 0
 * merges fine subdomains s into groups s * n_sub / n_fine first.  Empty
 * groups are dropped; each group grows by `overlap` layers of the coarse
 * graph.  Inner stopping: ||r|| < max(rtol ||b||, atol) or max_it
 * iterations (restart inner restart); a capped inner solve returns its
 * iterate and is counted.  The outer GMRES keeps its preconditioned
 * vectors (x = x0 + Z y), which is the flexible form (FGMRES) that a
 * preconditioner changing from one application to the next requires.
 * Allocates the coarse graph problem, its RAS and Krylov basis (device
 * memory) and selects coarse solver 2; the coarse data are formed by the
 * next seird_precond_setup.  Two-level preconditioners only; no transposed
 * form (SEIRD_ERR_ARG from a transposed apply).  Switching between the
 * direct solvers (0, 1) and 2 takes effect at the next setup (an apply in
 * between returns SEIRD_ERR_ARG). */
typedef struct {
  int32_t n_sub;    /* 0: one coarse subdomain per fine subdomain with coarse nodes */
  int32_t overlap;  /* layers of coarse-graph neighbours (1: minimal overlap) */
  int32_t restart;  /* inner GMRES restart, 1..31 */
  int32_t max_it;   /* inner iteration cap (100 in Section 3.2) */
  double rtol, atol;
} seird_coarse_krylov_opts;
seird_status seird_precond_set_coarse_krylov(seird_precond pc,
                                             const seird_coarse_krylov_opts *o);
typedef struct {
  int64_t solves;       /* inner solves since the last reset */
  int64_t its;          /* their iterations, summed */
  int64_t its_max;
  int64_t unconverged;  /* stopped by the cap (or the divergence test) */
  int32_t coarse_subdomains;
  int64_t coarse_local_unknowns;  /* summed over the coarse subdomains */
  int32_t amg_levels;             /* V3: levels of the AMG hierarchy */
  int64_t amg_last_nodes;         /* V3: nodes of its last level */
} seird_coarse_krylov_stats;
/* Two-grid RAS-V3 (Section 3.2): as V2, but the inner GMRES is
 * preconditioned by one V-cycle of algebraic multigrid on the coarse
 * system: plain aggregation of the coarse graph (greedy in the coarse
 * grid's node order: a node with no aggregated neighbour starts an
 * aggregate with its neighbours, the remaining nodes join the aggregate of
 * their lowest-numbered neighbour aggregated first, nodes still left start
 * aggregates with their free neighbours), piecewise-constant prolongation
 * per component, Galerkin block sums, until a level has at most max_coarse
 * nodes (or stops shrinking); nu damped (omega) node-block Jacobi sweeps
 * before and after each coarse correction, starting from zero; an explicit
 * dense inverse of the last level (Gaussian elimination with partial
 * pivoting at every setup; SEIRD_ERR_BREAKDOWN if singular).  The package
 * the paper uses (BoomerAMG) coarsens by classical splitting instead.
 * Selects coarse solver 3; allocates the hierarchy (device memory). */
typedef struct {
  int32_t max_coarse;  /* nodes of the last level, 1 .. 800 */
  int32_t nu;          /* smoothing sweeps before and after, 1 .. 8 */
  double omega;        /* Jacobi damping, (0, 2) */
  int32_t restart, max_it;
  double rtol, atol;
} seird_coarse_amg_opts;
seird_status seird_precond_set_coarse_amg(seird_precond pc,
                                          const seird_coarse_amg_opts *o);
seird_status seird_precond_coarse_krylov_stats(seird_precond pc,
                                               seird_coarse_krylov_stats *s,
                                               int reset);
/* Super-block size of the coarse inverses, in coarse tile rows (takes effect
 * at the next seird_precond_setup).  0: one block, the full inverses
 * X = L^{-1}, W = U^{-1} (the solve is two triangular mat-vecs).  Smaller
 * blocks shorten the setup (no inverse column recurrence is longer than a
 * block) and lengthen the solve (two steps per block).  Default 128, raised
 * to the coarse band width.  SEIRD_ERR_ARG when no inverses exist or the
 * size is below the coarse band width in tiles (the blocks must couple only
 * with their neighbours). */
seird_status seird_precond_set_coarse_block(seird_precond pc, int32_t tiles);
/* Workgroup size of the subdomain solves: 256 (any tile), 128, 512 or
 * 1024 (tile 32 only).  A launch choice: each row's sums are split over 4,
 * 8, 16 or 32 lanes (float64 accumulation), so results agree to rounding.
 * Default 256; SEIRD_ERR_ARG for other values. */
seird_status seird_precond_set_solve_threads(seird_precond pc, int32_t threads);

/* Autotuner of the Schwarz launch shapes on the caller's own problem: the
 * tile size of the factor storage (16 or 32; `opts->tile` is overridden) and
 * the subdomain-solve workgroup size.  For every tile it builds the
 * preconditioner from `opts` and `part`, factors `vals` twice (a warm-up,
 * then a host-timed setup), and for every workgroup size times `reps`
 * applications to a fixed vector with HIP events.  The score of a
 * candidate is setup_ms / applies_per_setup + apply_ms: the cost per
 * Krylov iteration when one setup serves applies_per_setup iterations.  A
 * candidate the problem does not admit (e.g. a band too wide for tile 16)
 * is reported with its status and skipped.  The candidate preconditioners
 * are destroyed before return (peak device memory: one preconditioner).
 * Synchronising; SEIRD_ERR_ARG if no candidate could be built. */
#define SEIRD_TUNE_MAX 8
typedef struct {
  int32_t tile, solve_threads;
  int32_t status; /* SEIRD_OK, or why the candidate was skipped */
  double setup_ms, apply_ms, score_ms;
} seird_tune_candidate;
typedef struct {
  int32_t best_tile, best_solve_threads;
  int32_t n_candidates;
  seird_tune_candidate cand[SEIRD_TUNE_MAX];
  int32_t from_cache;  /* 1: the choice came from the autotuner cache (no candidate timed) */
} seird_tune_report;
/* The autotuner cache: every choice of seird_autotune_schwarz and
 * seird_batch_autotune is kept per (device architecture, kernel, shape
 * bucket: nodes per subdomain in powers of two, overlap, one or two levels,
 * factor precision) for the process and, when the environment variable
 * SEIRD_TUNE_CACHE names a file, in that file; a later call with the same
 * key returns the kept choice without timing (from_cache = 1).  This call
 * empties the process's cache (the file is left alone and not read
 * again). */
seird_status seird_tune_cache_clear(void);
seird_status seird_autotune_schwarz(seird_problem p,
                                    const seird_schwarz_opts *opts,
                                    const int32_t *part, const double *vals,
                                    int32_t applies_per_setup, int32_t reps,
                                    seird_tune_report *report, void *stream);
/* Extract R_i A R_i^T from the Jacobian `vals`, factor every local matrix
 * (and the Galerkin coarse matrix) by LU without pivoting.  Synchronising;
 * returns SEIRD_ERR_BREAKDOWN on a zero/nonfinite pivot. */
seird_status seird_precond_setup(seird_precond pc, const double *vals,
                                 void *stream);
/* Setup of a compartment-wise (scalar) preconditioner, such as the one of
 * seird_pgs_precond, from a scalar matrix on the node graph: diag [n_nodes]
 * and off [n_slots] (slot order of seird_pattern), device float64.  Its
 * apply then maps vectors of n_nodes entries.  Synchronising;
 * SEIRD_ERR_BREAKDOWN on a zero or nonfinite pivot, SEIRD_ERR_ARG for a
 * coupled (node-block) preconditioner. */
seird_status seird_precond_setup_scalar(seird_precond pc, const double *diag,
                                        const double *off, void *stream);
/* z = M^{-1} r (transpose = 0) or M^{-T} r (transpose = 1), with M the
 * one-level RAS (Eq. RAS) or the multiplicative two-grid operator.  Async. */
seird_status seird_precond_apply(seird_precond pc, const double *r, double *z,
                                 int transpose, void *stream);

/* Solve J x = b (or J^T x = b) by right-preconditioned restarted GMRES.
 * `pc` may be NULL (no preconditioner).  Synchronising (stats). */
seird_status seird_gmres(seird_problem p, seird_precond pc, const double *vals,
                         const double *b, double *x,
                         const seird_krylov_opts *opts,
                         seird_krylov_stats *stats, int transpose,
                         void *stream);

/* Allocation-free GMRES, for callers that cannot allocate device memory
 * (serving loops with a fixed memory budget, harnesses that forbid
 * hipMalloc during a run).  The same solve as seird_gmres, with the same
 * arguments, kernels and results, except that its scratch -- the Krylov
 * basis V [restart+1][N], the preconditioned vectors Z [restart][N], the
 * reduction partials and the Arnoldi coefficients -- lives in a fixed
 * device array of SEIRD_STATIC_SCRATCH_BYTES compiled into the library:
 * one per GPU, held from the library's first use on that GPU until the
 * process ends.  The call allocates no device memory (the problem and
 * the preconditioner were created beforehand; the problem's pinned staging
 * buffer is reserved at its creation), and HIP graphs are not used
 * (opts->graphs is ignored).  Limits: (2 restart + 1) * N * 8 bytes plus a
 * few KB must fit the array, else SEIRD_ERR_ARG (N = 5 n_nodes; restart 30
 * admits about 137k unknowns); a single problem (not a batch's);
 * preconditioner timing must be off (SEIRD_ERR_ARG).  Every call on one GPU
 * shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (other host threads, other streams) race and must be
 * serialised by the caller.  Synchronising, like seird_gmres. */
#define SEIRD_STATIC_SCRATCH_BYTES (64LL << 20)
seird_status seird_gmres_noalloc(seird_problem p, seird_precond pc,
                                 const double *vals, const double *b,
                                 double *x, const seird_krylov_opts *opts,
                                 seird_krylov_stats *stats, int transpose,
                                 void *stream);

/* One implicit step: u (in: u^n, out: u^{n+1}).  Newton iterations: F,
 * J, preconditioner setup, GMRES, update.  Synchronising.  On failure u is
 * unspecified and stats->reason holds the status. */
seird_status seird_step(seird_problem p, seird_precond pc, double *u,
                        double dt, const double *src,
                        const seird_newton_opts *nopts,
                        const seird_krylov_opts *kopts,
                        seird_step_stats *stats, void *stream);

/* ------------------------------------------------------------------
 * Decoupled Picard-Gauss-Seidel step (the paper's own nonlinear solver,
 * Section 2.2 Eq. weak_vec_implicit with the per-compartment weak forms of
 * Appendix A and the stopping rule of Eq. picardtol).  A sweep lags the
 * diffusion coefficient N and the Allee factor (1 - A/N) at the sweep's
 * start and solves the compartments S, E, I, R, D one after the other as
 * scalar systems on the node graph (lumped mass, exact P1 diffusion with
 * the element-mean lagged density), each using the compartments already
 * updated in the sweep; vital dynamics enter as loss rate mu on the
 * diagonal and birth alpha N (lagged) on the right-hand side.  Each system
 * is solved in correction form, A_c delta = rhs_c - A_c u_c, by GMRES with a
 * one-level RAS over scalar subdomains (a compartment with nu_c = 0 is
 * diagonal and is solved directly).  The sweeps stop when
 * epsilon = ||u^{k+1} - u^k||_2 / ||u^n||_2 <= tol.  The fixed point is the
 * root of the coupled residual that seird_step reaches (only the iteration
 * differs); res_scaled reports ||F(u)||_2 / ||M_L u^n||_2 at the result.
 * ------------------------------------------------------------------ */
typedef struct seird_pgs_s *seird_pgs;
#define SEIRD_MAX_PGS 64
typedef struct {
  double tol;          /* epsilon tolerance of Eq. picardtol */
  int32_t max_sweeps;  /* 1 .. SEIRD_MAX_PGS */
  int32_t strict_linear; /* 1: a GMRES solve stopping at max_it fails the step */
  /* 1: each diffusing compartment's preconditioner is set up at the first
   * sweep of the step and kept for its later sweeps (one setup per
   * compartment and step; each compartment then holds its own factors);
   * 0: a setup before every solve.  The fixed point does not depend on it,
   * only the GMRES counts do.  seird22_step ignores it (its preconditioners
   * are kept by design). */
  int32_t pc_lag;
} seird_pgs_opts;
typedef struct {
  int32_t sweeps;
  int32_t gmres_its[5];      /* per compartment, summed over the sweeps */
  double eps_hist[SEIRD_MAX_PGS];
  double res_scaled;         /* coupled residual of the result, scaled */
  int32_t pc_setups, inexact_solves;
  int32_t reason;
  double t_setup_ms, t_gmres_ms, t_total_ms;
} seird_pgs_stats;
/* The solver of problem p with scalar subdomains from the partition and
 * opts (n_sub, overlap, tile, factor_prec; n_ref must be 0).  Device work
 * arrays are allocated here. */
seird_status seird_pgs_create(seird_problem p, const seird_schwarz_opts *opts,
                              const int32_t *part, seird_pgs *out);
void seird_pgs_destroy(seird_pgs g);
/* Its scalar preconditioner, borrowed (seird_precond_info / _timing /
 * _set_solve_threads). */
seird_status seird_pgs_precond(seird_pgs g, seird_precond *out);
/* One implicit step by Picard-Gauss-Seidel sweeps, u in: u^n, out: u^{n+1}.
 * Synchronising.  SEIRD_ERR_NOT_CONVERGED when max_sweeps do not reach tol;
 * on failure u is unspecified and stats->reason holds the status. */
seird_status seird_pgs_step(seird_pgs g, double *u, double dt,
                            const seird_pgs_opts *popts,
                            const seird_krylov_opts *kopts,
                            seird_pgs_stats *stats, void *stream);

/* ------------------------------------------------------------------
 * Batches: several independent problems (uneven meshes, their own rates
 * and diffusion coefficients) stepped together.  The instances are laid
 * side by side as one block-diagonal system, so every kernel (assembly,
 * SpMV, every Schwarz subdomain factorisation and solve, in
 * largest-first order) is one launch over all instances, while every
 * reduction, GMRES coefficient, stopping test and Newton iteration is kept
 * per instance: each instance's result is the one it gets alone (bitwise
 * for pc_reuse = 0).  One-level RAS.
 * ------------------------------------------------------------------ */
typedef struct seird_batch_s *seird_batch;
/* n_inst instances; per instance k: n_nodes[k], xy[k] (host [n][2]),
 * n_tri[k], tri[k] (host [n_tri][3], local numbering), params[k],
 * part[k] (host [n_nodes[k]] owner subdomain in [0, n_sub[k])).  overlap,
 * tile and factor_prec as in seird_schwarz_opts.  Host arrays are copied. */
seird_status seird_batch_create(int32_t n_inst, const int64_t *n_nodes,
                                const double *const *xy,
                                const int64_t *n_tri,
                                const int32_t *const *tri,
                                const seird_params *params,
                                const int32_t *const *part,
                                const int32_t *n_sub, int32_t overlap,
                                int32_t tile, int32_t factor_prec,
                                seird_batch *out);
void seird_batch_destroy(seird_batch b);
/* node_offsets [n_inst + 1] (host): instance k owns nodes
 * [node_offsets[k], node_offsets[k+1]) of the batch state. */
seird_status seird_batch_info(seird_batch b, int64_t *node_offsets);
/* Autotune the subdomain-solve width of the batch's preconditioner on the
 * ensemble itself (its current factors: call after a step): times `reps`
 * subdomain-solve launches over every instance for each width (256, 128,
 * 512, 1024 with tile 32), keeps the fastest (also in the autotuner cache).
 * Synchronising. */
seird_status seird_batch_autotune(seird_batch b, int32_t reps, seird_tune_report *report,
                                  void *stream);
/* The batch's preconditioner (one-level RAS over the subdomains of every
 * instance), borrowed: owned by the batch and valid until
 * seird_batch_destroy.  For seird_precond_timing / seird_precond_info. */
seird_status seird_batch_precond(seird_batch b, seird_precond *out);
/* One implicit step of every instance: u is the device float64 state
 * [total_nodes][5], instance after instance.  per_instance[n_inst]
 * (nullable) receives each instance's Newton/GMRES statistics.
 * Synchronising. */
seird_status seird_batch_step(seird_batch b, double *u, double dt,
                              const seird_newton_opts *nopts,
                              const seird_krylov_opts *kopts,
                              seird_step_stats *per_instance, void *stream);

/* ------------------------------------------------------------------
 * Discrete adjoint of a case-count observation (reverse sweep with
 * checkpointing).  Parameters theta = (g, nu): the transmission field g
 * (seird_set_beta_field) and the five diffusion coefficients nu
 * (seird_params).  Observation: c_r^n = sum_{j in r} m_j i_j^n for regions
 * r = 0..n_regions-1 and steps n = 1..n_steps.  With lam^n solving
 *   J_n^T lam^n = dL/du^n + M lam^{n+1}   (J_n = dF^n/du^n, lam^{N+1} = 0),
 * the gradient of a loss L(c) is dL/dtheta = - sum_n (dF^n/dtheta)^T lam^n.
 * ------------------------------------------------------------------ */
typedef struct {
  int32_t gmres_its_total;  /* transposed solves */
  int32_t recomputed_steps;
  double t_forward_ms, t_reverse_ms;
  int32_t setups;           /* preconditioner setups of the transposed solves */
} seird_adjoint_stats;

/* Run n_steps implicit steps from u (in: u^0, out: u^{n_steps}), record
 * checkpoints every ckpt_every steps (device memory owned by the problem;
 * replaces any previous record) and write the counts [n_steps][n_regions]
 * (device float64).  The states of the last checkpoint segment are kept
 * as well: with ckpt_every >= n_steps every state stays in device memory
 * (ckpt_every + 1 state vectors) and seird_adjoint recomputes no step.
 * region: host int32 [n_nodes], -1 = unobserved.  Synchronising. */
seird_status seird_forward_record(seird_problem p, seird_precond pc,
                                  double *u, int32_t n_steps, double dt,
                                  int32_t ckpt_every, const int32_t *region,
                                  int32_t n_regions, double *counts,
                                  const seird_newton_opts *nopts,
                                  const seird_krylov_opts *kopts,
                                  void *stream);
/* Reverse sweep of the last record: grad_counts [n_steps][n_regions]
 * (device, dL/dc), outputs grad_g [n_nodes] (device) and grad_nu [5]
 * (host).  Transposed solves use GMRES with the transposed preconditioner
 * (kopts).  Parameters must be those of the record.  Synchronising. */
seird_status seird_adjoint(seird_problem p, seird_precond pc,
                           const double *grad_counts, double *grad_g,
                           double *grad_nu, const seird_krylov_opts *kopts,
                           seird_adjoint_stats *stats, void *stream);

/* ------------------------------------------------------------------
 * The 22-compartment model of Appendix C (Eqs. S ... D).  Compartments in
 * the order of its compartment table, node-major state [n][22]:
 *   S V E Q A W F B C X Y Z G N H H1 I H2 R1 R2 P D   (indices 0 .. 21);
 * S V E A F B C P R1 R2 diffuse with constant coefficients nu[0..9] (in
 * that order), the others are nodal.  Backward Euler with the lumped mass
 * and homogeneous Neumann data of the five-compartment path:
 *   F_c(u) = m (u_c - u_c^n) + dt nu_c K u_c - dt m R_c(u) = 0.
 * The force of infection, which Appendix C uses but does not define, is
 * lambda = beta_A A + beta_F F + beta_B B + beta_C C (mass action in the
 * moving, non-isolating infectious densities, as in Eqs. seird1-5); phi_C
 * of the equations is the parameter the table calls phi_A.
 * ------------------------------------------------------------------ */
#define SEIRD22_NC 22
typedef struct {
  double beta_A, beta_F, beta_B, beta_C;
  double r_V, delta_S, delta_V;
  double gamma_A, gamma_C, gamma_DA, gamma_DM, gamma_E, gamma_I, gamma_L,
      gamma_M, gamma_P, gamma_R, gamma_S1, gamma_S2, gamma_T, gamma_V;
  double sigma_A, sigma_C, sigma_H, sigma_S;
  double pi_A, pi_B, pi_C, pi_H;
  double phi_C, phi_M, phi_S, phi_P;
  double kappa_H, kappa_I, kappa_N, kappa_P;
  double nu[10]; /* S V E A F B C P R1 R2 */
} seird22_params;
typedef struct seird22_s *seird22;
/* A 22-compartment problem on a mesh handle, stepped by the decoupled
 * Picard-Gauss-Seidel iteration of Appendix A applied compartment by
 * compartment: every reaction term is affine in its own density,
 * R_c = s_c - d_c u_c, so a sweep solves, in table order and with the
 * latest densities of the others, (m (1 + dt d_c) + dt nu_c K) u_c =
 * m u_c^n + dt m s_c: a diagonal division for the twelve nodal
 * compartments, and for the ten diffusing ones GMRES with a one-level RAS
 * of scalar subdomains (opts: n_sub, overlap, tile; one-level, FP64) built
 * from part.  The preconditioner of a compartment whose d_c does not depend
 * on the state (all but S and V) is set up once per time-step size; those
 * of S and V at the first sweep of every step.  Allocates device memory. */
seird_status seird22_create(seird_mesh mesh, const seird22_params *p,
                            const seird_schwarz_opts *opts,
                            const int32_t *part, seird22 *out);
void seird22_destroy(seird22 h);
seird_status seird22_set_params(seird22 h, const seird22_params *p);
/* F [n][22] = the residual above at u (device [n][22]) with u^n = u_prev. */
seird_status seird22_residual(seird22 h, const double *u, const double *u_prev,
                              double dt, double *F, void *stream);
typedef struct {
  int32_t sweeps;
  int32_t gmres_its[SEIRD22_NC]; /* per compartment, summed over the sweeps */
  double eps_hist[SEIRD_MAX_PGS];  /* ||u^{k+1} - u^k|| / ||u^n|| */
  double res_scaled;               /* ||F(u)|| / ||m u^n|| of the result */
  int32_t pc_setups, inexact_solves;
  int32_t reason;
  double t_setup_ms, t_gmres_ms, t_total_ms;
} seird22_stats;
/* One step in place on u (device [n][22]).  Sweeps until epsilon <= tol
 * (SEIRD_ERR_NOT_CONVERGED after max_sweeps); kopts: the inner GMRES.
 * SEIRD_ERR_NONFINITE for a nonfinite state.  Synchronising. */
seird_status seird22_step(seird22 h, double *u, double dt,
                          const seird_pgs_opts *popts,
                          const seird_krylov_opts *kopts,
                          seird22_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SEIRD_H */
