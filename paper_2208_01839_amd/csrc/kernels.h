// Launch interface between the host orchestration and the HIP kernels.
#pragma once

#include "internal.h"

namespace seird {

constexpr int KRYLOV_MAX = 32;  // max basis vectors handled by one Arnoldi kernel
// size of the per-device static scratch of the allocation-free entry points
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)SEIRD_STATIC_SCRATCH_BYTES;
// device address of this device's static scratch (looked up once per
// device, with that device current; valid until the process ends)
void *static_scratch();
constexpr int SEG_CH = 1024;    // entries per block of a segmented reduction

struct SegView;
// Segments of a vector (instances of a batch; one segment for a single
// problem) and their reduction blocks, on host and device.
struct SegHost {
  int S = 0, B = 0;
  std::vector<int64_t> seg_start, blk_start;
  std::vector<int32_t> block_seg;
  int64_t *d_seg_start = nullptr, *d_blk_start = nullptr;
  int32_t *d_block_seg = nullptr;
  uint8_t *d_active = nullptr;  // nullable: all active
  SegView view() const;
};

struct FactorLaunch {
  int tile = 32;
  int bs = 5;               // unknowns per node of the extracted matrix (5: node-block Jacobian; 1: scalar)
  bool dense_off = false;   // bs 5 with dense off-diagonal blocks, off [slots][25] (the coarse graph matrix)
  void *Fs = nullptr;       // subdomain tile-envelope storage (float64, or float32 if sub_float)
  bool sub_float = false;   // factorise the subdomains in float32
  void *Fh = nullptr;       // with sub_float and tile 32: also write each final factor entry here in bfloat16
  int64_t sub_entries = 0;
  double *Fc = nullptr;     // coarse tile-band storage (float64)
  int64_t coarse_entries = 0;
  const SubInfo *subs = nullptr;  // device
  const int32_t *erow = nullptr, *elo = nullptr;  // subdomain row tables (device)
  int nsub = 0;
  const int32_t *order = nullptr;
  const ExtractEntry *ent = nullptr;  // grouped by (subdomain, local node)
  const int32_t *ent_ptr = nullptr;   // first entry of each local node
  const int32_t *trow_ptr = nullptr;  // first global tile row of each subdomain [nsub+1]
  const int32_t *trow_sub = nullptr;  // subdomain of each global tile row [ntrows]
  int64_t ntrows = 0;                 // tile rows over all subdomains
  int max_node_blocks = 0;            // most extraction entries of one local node
  int max_bu = 0;
  int *status = nullptr;
  // persistent factorisation grid: queue counter (device int), compute
  // units, and workgroup slots left for the concurrent coarse chain
  int *queue = nullptr;
  int n_cu = 0;
  int lu_spare = 32;
  // coarse
  bool coarse = false;
  SubInfo cs{};
  const SubInfo *coarse_dev = nullptr;
  const int32_t *gp = nullptr, *gq = nullptr;
  const int64_t *gptr = nullptr;
  const int32_t *gref = nullptr;
  const double *gw = nullptr;
  int64_t gal_nblk = 0;
  // optional timing events on st: before the extraction, between the
  // extraction and the subdomain factorisation, after the factorisation
  hipEvent_t ev_extract = nullptr, ev_lu = nullptr, ev_lu_end = nullptr;
};

struct SolveLaunch {
  int tile = 32;
  int prec = 0;
  const void *F = nullptr;
  const SubInfo *subs = nullptr;
  const int32_t *erow = nullptr, *elo = nullptr;  // row tables of envelope-layout systems
  const int32_t *order = nullptr;
  int nblocks = 0;
  bool wide = false;  // 1024-thread workgroups (one large system)
  int threads = 256;  // workgroup size of the subdomain solves (256; 512, 1024 for tile 32)
  const int32_t *l2g = nullptr;
  const uint8_t *owned = nullptr;
  const double *r = nullptr;
  double *z = nullptr;
  int add = 0;
  int transpose = 0;
  double *yloc = nullptr;
  double *ybuf = nullptr;  // forward-sweep results, sum of n_loc (or coarse n_loc) doubles
  // optional: instance of every subdomain and the active flag of every
  // instance; subdomains of inactive instances are skipped
  const int32_t *sub_seg = nullptr;
  const uint8_t *seg_active = nullptr;
};

void launch_residual(const MeshDev &m, const ParamsDev &P, const double *g, const double *u, const double *up,
                     double dt, const double *src, double *F, hipStream_t st);
void launch_jacobian(const MeshDev &m, const ParamsDev &P, const double *g, const double *u, double dt, double *diag,
                     double *off, hipStream_t st);
void launch_spmv(const MeshDev &m, const double *diag, const double *off, const double *x, const double *b, double *y,
                 int transpose, hipStream_t st);
void launch_mdot(const double *V, int64_t ldv, int nv, const double *w, int64_t N, int with_self, double *partials,
                 int nb, hipStream_t st);
void launch_reduce(const double *partials, int nb, int nv, double *out, hipStream_t st);
void launch_maxpy_norm(double *w, const double *V, int64_t ldv, const double *h, int nv, int64_t N, double *partials,
                       int nb, hipStream_t st);
void launch_gemv_update(double *x, const double *Z, int64_t ldz, const double *y, int nv, int64_t N, int nb,
                        hipStream_t st);
void launch_fill(double *y, double v, int64_t N, hipStream_t st);
void launch_fill_int(int *y, int v, int N, hipStream_t st);
void launch_axpby(double *y, const double *x, double a, const double *aptr, int ainv, double b, int64_t N, int nb,
                  hipStream_t st);
void launch_norm2_partials(const double *x, const double *scale, int64_t N, double *partials, int nb, hipStream_t st);
// scalar CSR values of the node-block Jacobian (pattern of seird_csr)
void launch_csr_values(const MeshDev &m, const double *diag, const double *off, const int64_t *csr_rowptr,
                       double *out, hipStream_t st);
// decoupled Picard-Gauss-Seidel sweep: lagged scalar stiffness, one
// compartment's scalar system (correction form), scalar SpMV, update
void launch_pgs_stiffness(const MeshDev &m, const double *uk, double *Kd, double *Ko, hipStream_t st);
void launch_pgs_system(const MeshDev &m, const ParamsDev &P, const double *g, int c, double dt, const double *u,
                       const double *uk, const double *un, const double *Kd, const double *Ko, double *sdiag,
                       double *soff, double *r, hipStream_t st);
void launch_scalar_spmv(const MeshDev &m, const double *sdiag, const double *soff, const double *x, const double *b,
                        double *y, hipStream_t st);
void launch_pgs_update(double *u, int c, const double *delta, const double *sdiag, int64_t n, hipStream_t st);
// per-instance flags (inst nullable: one instance), flags[S] zeroed by the caller
void launch_check_state(const double *u, int64_t n, const int32_t *inst, int *flags, hipStream_t st);
// the coarse factorisation goes to st_coarse (may equal st), the subdomains to st
void launch_setup_factors(const FactorLaunch &fl, const double *diag, const double *off, hipStream_t st,
                          hipStream_t st_coarse);
// Galerkin coarse matrix as dense 5x5 node blocks of the coarse graph
// (block k to the diagonal block -gdst[k]-1 or to slot gdst[k])
void launch_galerkin_blocks(const int32_t *gdst, const int64_t *gptr, const int32_t *gref, const double *gw,
                            int64_t nblk, const double *diag, const double *off, double *cdiag, double *coff,
                            hipStream_t st);
// y = A x (b null) or b - A x for dense 5x5 node blocks: diag [n][25], off [slots][25]
void launch_block_spmv(int64_t n, const int64_t *rowptr, const int32_t *col, const double *diag, const double *off,
                       const double *x, const double *b, double *y, hipStream_t st);
// 22-compartment model (Appendix C), state [n][22]
void launch22_residual(const MeshDev &m, const seird22_params &p, const double *u, const double *up, double dt,
                       double *F, hipStream_t st);
void launch22_stiffness(const MeshDev &m, double *Kd, double *Ko, hipStream_t st);
void launch22_system(const MeshDev &m, const seird22_params &p, int c, double dt, double *u, const double *up,
                     const double *Kd, const double *Ko, double *sdiag, double *r, hipStream_t st);
void launch22_offdiag(int64_t ns, double coef, const double *Ko, double *soff, hipStream_t st);
void launch22_update(double *u, int c, const double *delta, int64_t n, hipStream_t st);
void launch22_mass_scale(const double *mass, const double *x, double *y, int64_t n, hipStream_t st);
void launch22_check(const double *u, int64_t N, int *flags, hipStream_t st);
// aggregation AMG over dense 5x5 node blocks: Galerkin sums of dense blocks
// (weights 1), diagonal-block inverses (*status |= 1 if singular), damped
// block Jacobi x += omega D^{-1} r, restriction / prolongation over the
// aggregates, dense matrix-vector product of the last level
void launch_galerkin_dense(const int32_t *gdst, const int64_t *gptr, const int32_t *gref, int64_t nblk,
                           const double *diag, const double *off, double *cdiag, double *coff, hipStream_t st);
void launch_block_inv5(int64_t n, const double *diag, double *dinv, int *status, hipStream_t st);
void launch_block_jacobi(int64_t n, const double *dinv, const double *r, double omega, double *x, hipStream_t st);
void launch_agg_restrict(int64_t nagg, const int64_t *agg_ptr, const int32_t *agg_nodes, const double *r, double *bc,
                         hipStream_t st);
void launch_agg_prolong(int64_t n, const int32_t *agg, const double *xc, double *x, hipStream_t st);
void launch_dense_gemv(int m, const double *M, const double *b, double *y, hipStream_t st);
void launch_convert(void *dst, int dst_prec, const void *src, int src_float, int64_t N, hipStream_t st);
void launch_band_solve(const SolveLaunch &sl, hipStream_t st);
void launch_gather_copies(const int64_t *gptr, const int32_t *gidx, const double *yloc, double *z, int add, int64_t N,
                          hipStream_t st);
void launch_coarse_restrict(const int64_t *zt_ptr, const int32_t *zt_col, const double *zt_val, const int32_t *cperm,
                            const double *r, double *rc, int64_t nc, hipStream_t st);
void launch_coarse_prolong(const int64_t *z_ptr, const int32_t *z_col, const double *z_val, const int32_t *cperm,
                           const double *xc, double *z, int64_t n, hipStream_t st);

void launch_region_counts(const int64_t *reg_ptr, const int32_t *reg_nodes, const double *mass, const double *u,
                          double *counts, int n_regions, hipStream_t st);
void launch_adjoint_rhs(const MeshDev &m, const int32_t *region, const double *gc, const double *lam_next,
                        double *rhs, hipStream_t st);
// returns the number of blocks (nu partial sums per component)
int launch_adjoint_grad(const MeshDev &m, const ParamsDev &P, const double *u, const double *lam, double dt,
                        double *grad_g, double *partials, hipStream_t st);

// one large band system (coarse, FP64, tile 32, bl, bu <= 16), non-transposed
void launch_coarse_solve(const double *F, const SubInfo *sp, const double *r, double *z, double *ybuf,
                         hipStream_t st);
// inverses X_II = L_II^{-1}, W_II = U_II^{-1} of the diagonal super-blocks
// of S tile rows of the factored coarse band (tile 32), packed triangular
// tile storage block after block (at most nt(nt+1)/2 tiles each)
void launch_coarse_inverse(const double *F, const SubInfo &cs, int S, double *X, double *W, hipStream_t st);
// coarse solve z = A_c^{-1} r (or A_c^{-T} r) by the block sweep over those
// super-blocks; r (overwritten), z, tmp: nt * 32 doubles
void launch_coarse_inverse_apply(const double *X, const double *W, const double *F, const SubInfo &cs, int S,
                                 double *r, double *z, double *tmp, double *part, int transpose, hipStream_t st);
// partial-sum slots (of 32 doubles) that one triangular mat-vec over a block
// of nt tile rows uses
int64_t coarse_tri_chunks(int nt);

void launch_seg_mdot(const SegHost &g, const double *V, int64_t ldv, int nv, const double *w, int with_self,
                     double *partials, hipStream_t st);
void launch_seg_reduce(const SegHost &g, const double *partials, int nrows, double *out, int ldo, int row_off,
                       hipStream_t st);
void launch_seg_maxpy_norm(const SegHost &g, double *w, const double *V, int64_t ldv, const double *h, int ldh, int nv,
                           double *partials, hipStream_t st);
void launch_seg_gemv_update(const SegHost &g, double *x, const double *Z, int64_t ldz, const double *y, int ldy, int nv,
                            hipStream_t st);
void launch_seg_axpby(const SegHost &g, double *y, const double *x, const double *a, double b, hipStream_t st);
void launch_seg_norm2(const SegHost &g, const double *x, const double *scale, double *partials, hipStream_t st);

}  // namespace seird
