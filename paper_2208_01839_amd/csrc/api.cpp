// C ABI of libseird and the host orchestration: Newton time step, restarted
// right-preconditioned GMRES, one-level and two-grid Schwarz apply.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <cstdio>
#include <functional>
#include <map>
#include <mutex>
#include <memory>
#include <tuple>

#include "kernels.h"

using namespace seird;

namespace seird {
static thread_local std::string g_last_error;
[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }
void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(SEIRD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
// caller workspaces in use: (base, bytes, handles referring to it)
struct WsEntry {
  uintptr_t base;
  size_t bytes;
  int refs;
};
static std::mutex g_ws_mu;
static std::vector<WsEntry> g_workspaces;
void register_workspace(const void *base, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  for (auto &w : g_workspaces)
    if (w.base == (uintptr_t)base) {
      w.refs++;
      return;
    }
  g_workspaces.push_back({(uintptr_t)base, bytes, 1});
}
void unregister_workspace(const void *base) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  for (size_t k = 0; k < g_workspaces.size(); ++k)
    if (g_workspaces[k].base == (uintptr_t)base) {
      if (--g_workspaces[k].refs == 0) g_workspaces.erase(g_workspaces.begin() + k);
      return;
    }
}
Arena *&active_arena() {
  static thread_local Arena *a = nullptr;
  return a;
}
bool measuring() { return active_arena() && active_arena()->measure; }
void *Arena::take(size_t bytes) {
  const size_t b = (bytes + 255) & ~(size_t)255;
  if (!measure && used + b > cap)
    fail(SEIRD_ERR_WORKSPACE, "workspace exhausted: " + std::to_string(used + b) + " bytes needed, " +
                                  std::to_string(cap) + " given");
  void *p = base + used;
  used += b;
  return p;
}
static std::atomic<int64_t> g_dev_allocs{0}, g_dev_alloc_bytes{0};
void *dev_alloc_bytes(size_t bytes) {
  if (Arena *a = active_arena()) return a->take(bytes);
  void *p = nullptr;
  HIPCHECK(hipMalloc(&p, bytes));
  g_dev_allocs++;
  g_dev_alloc_bytes += (int64_t)bytes;
  return p;
}
void dev_free(void *p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    for (const auto &w : g_workspaces)
      if ((uintptr_t)p >= w.base && (uintptr_t)p < w.base + w.bytes) return;
  }
  (void)hipFree(p);
}
}  // namespace seird

#define API_BEGIN try {
#define API_END                                   \
  }                                               \
  catch (const Error &e) {                        \
    g_last_error = e.msg;                         \
    return e.code;                                \
  }                                               \
  catch (const std::exception &e) {               \
    g_last_error = std::string("internal: ") + e.what(); \
    return SEIRD_ERR_ARG;                         \
  }                                               \
  return SEIRD_OK;

static ParamsDev to_dev(const seird_params &p) {
  ParamsDev d{};
  d.sigma = p.sigma; d.gE = p.gamma_E; d.gR = p.gamma_R; d.gD = p.gamma_D;
  d.A = p.A; d.alpha = p.alpha; d.mu = p.mu; d.bI = p.beta_I; d.bE = p.beta_E;
  for (int c = 0; c < 5; ++c) d.nu[c] = p.nu[c];
  return d;
}

static int reduction_blocks(int64_t N) {
  int64_t nb = (N + 4 * 256 - 1) / (4 * 256);
  return (int)std::max<int64_t>(1, std::min<int64_t>(nb, 2048));
}

struct seird_problem_s {
  int device = 0;
  MeshHost mh;
  MeshDev md;
  ParamsDev P{};
  double *gfield = nullptr;
  int64_t N = 0;      // unknowns
  int nb = 1;         // reduction grid
  // transmission schedule (Eq. beta_ie): beta_I and beta_E are multiplied
  // by a - b / (1 + exp(k (tc - t))) at the time the coefficients refer to
  bool sched = false;
  double sa = 0.0, sb = 0.0, sk = 0.0, stc = 0.0;
  double time = 0.0;  // model time of the current state
  ParamsDev params_at(double t) const {
    ParamsDev q = P;
    if (sched) {
      const double f = sa - sb / (1.0 + std::exp(sk * (stc - t)));
      q.bI *= f;
      q.bE *= f;
    }
    return q;
  }
  // discretisation variants: consistent-mass values and the stored
  // boundary flux field (always allocated; md points at them when enabled)
  double *d_cmass_d = nullptr, *d_cmass_o = nullptr, *d_qflux = nullptr;
  int64_t *d_bnd_ptr = nullptr;
  int32_t *d_bnd_j = nullptr;
  double *d_bnd_nl = nullptr;
  double *partials = nullptr;
  double *hdev = nullptr;   // small device vector (Arnoldi coefficients, norms)
  double *ydev = nullptr;
  int *flags = nullptr;
  // Newton work
  double *u_prev = nullptr, *F = nullptr, *rhs = nullptr, *delta = nullptr, *vals = nullptr;
  // Krylov basis
  double *V = nullptr, *Zb = nullptr;
  int kcap = 0;
  double *w1 = nullptr;  // scratch vector
  size_t lds_limit = 65536;
  int n_cu = 0;  // compute units of the device
  // segments of the unknown vector (one per instance of a batch; one for a
  // single problem), per-segment masks and scalars
  static constexpr int HLD = KRYLOV_MAX + 8;
  SegHost seg, seg_act, seg_re;  // no mask / active mask / second mask
  uint8_t *d_mask = nullptr, *d_mask2 = nullptr;
  double *d_svec = nullptr;
  int32_t *d_inst = nullptr;
  ParamsDev *d_Pinst = nullptr;
  // caller workspace (seird_create_in_workspace), else null: device
  // memory then comes from it only, with the Krylov basis reserved for
  // ws_restart, a stored transmission field and a pool for adjoint records
  void *ws_base = nullptr;
  size_t ws_bytes = 0;
  int ws_restart = 0;
  Arena tape_pool;
  double *gfield_store = nullptr;
  // scalar CSR pattern of the Jacobian (seird_csr), built on first request
  int64_t *csr_rowptr = nullptr;
  int32_t *csr_col = nullptr;
  int64_t csr_nnz = 0;
  bool csr_reserved = false;  // workspace problems: room kept at creation
  void build_csr() {
    const int64_t n = mh.n;
    std::vector<int64_t> rp(5 * n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t deg = mh.rowptr[i + 1] - mh.rowptr[i];
      for (int c = 0; c < 5; ++c) rp[5 * i + c + 1] = rp[5 * i + c] + 5 * (deg + 1);
    }
    std::vector<int32_t> col(rp[5 * n]);
    for (int64_t i = 0; i < n; ++i) {
      std::vector<int32_t> nodes(mh.col.begin() + mh.rowptr[i], mh.col.begin() + mh.rowptr[i + 1]);
      nodes.insert(std::lower_bound(nodes.begin(), nodes.end(), (int32_t)i), (int32_t)i);
      for (int c = 0; c < 5; ++c) {
        int64_t q = rp[5 * i + c];
        for (int32_t j : nodes)
          for (int cp = 0; cp < 5; ++cp) col[q++] = 5 * j + cp;
      }
    }
    csr_nnz = rp[5 * n];
    if (csr_rowptr) {  // reserved in the workspace: fill in place
      HIPCHECK(hipMemcpy(csr_rowptr, rp.data(), sizeof(int64_t) * rp.size(), hipMemcpyHostToDevice));
      HIPCHECK(hipMemcpy(csr_col, col.data(), sizeof(int32_t) * col.size(), hipMemcpyHostToDevice));
    } else {
      csr_rowptr = dev_upload(rp);
      csr_col = dev_upload(col);
    }
  }
  bool csr_ready = false;
  // adjoint record (checkpoints, last segment, regions)
  struct Tape {
    int n_steps = 0, every = 0, n_regions = 0;
    double dt = 0.0, t0 = 0.0;  // step size, model time of the first state
    seird_newton_opts nopts{};
    seird_krylov_opts kopts{};
    std::vector<double *> ckpt, seg;
    int seg_holds = -1;  // index of the segment whose states T.seg holds
    int32_t *region = nullptr, *reg_nodes = nullptr;
    int64_t *reg_ptr = nullptr;
    double *lam = nullptr, *lam_next = nullptr, *rhs = nullptr, *partials = nullptr;
    bool valid = false;
    void release() {
      for (double *q : ckpt) dev_free(q);
      for (double *q : seg) dev_free(q);
      ckpt.clear();
      seg.clear();
      dev_free(region); dev_free(reg_nodes); dev_free(reg_ptr);
      dev_free(lam); dev_free(lam_next); dev_free(rhs); dev_free(partials);
      region = reg_nodes = nullptr;
      reg_ptr = nullptr;
      lam = lam_next = rhs = partials = nullptr;
      seg_holds = -1;
      valid = false;
    }
  } tape;
  // the arena of adjoint-record allocations (null: hipMalloc)
  Arena *tape_arena() { return ws_base ? &tape_pool : nullptr; }
  void release_tape() {
    tape.release();
    tape_pool.used = 0;
  }

  ~seird_problem_s() {
    dev_free(md.rowptr); dev_free(md.col); dev_free(md.tslot); dev_free(md.mass);
    dev_free(md.inc_ptr); dev_free(md.inc_j); dev_free(md.inc_l); dev_free(md.inc_sj); dev_free(md.inc_sl);
    dev_free(md.slot_row); dev_free(md.slot_ek); dev_free(md.kd); dev_free(md.ko); dev_free(md.kw);
    dev_free(md.inc_K);
    dev_free(gfield); dev_free(partials); dev_free(hdev); dev_free(ydev); dev_free(flags);
    dev_free(u_prev); dev_free(F); dev_free(rhs); dev_free(delta); dev_free(vals);
    dev_free(V); dev_free(Zb); dev_free(w1);
    dev_free(seg.d_seg_start); dev_free(seg.d_blk_start); dev_free(seg.d_block_seg);
    dev_free(d_mask); dev_free(d_mask2); dev_free(d_svec); dev_free(d_inst); dev_free(d_Pinst);
    dev_free(csr_rowptr); dev_free(csr_col);
    dev_free(d_cmass_d); dev_free(d_cmass_o); dev_free(d_qflux); dev_free(d_bnd_ptr); dev_free(d_bnd_j);
    dev_free(d_bnd_nl);
    tape.release();
    if (stage) {
      (void)hipStreamSynchronize(stage_st);
      (void)hipHostFree(stage);
    }
    if (dl) (void)hipHostFree(dl);
    if (ws_base) unregister_workspace(ws_base);
  }

  // segments from instance node offsets (node_start[S+1], node_start[S] = n)
  void setup_segments(const std::vector<int64_t> &node_start) {
    dev_free(seg.d_seg_start); dev_free(seg.d_blk_start); dev_free(seg.d_block_seg);
    SegHost g;
    g.S = (int)node_start.size() - 1;
    g.seg_start.resize(g.S + 1);
    g.blk_start.assign(g.S + 1, 0);
    for (int s = 0; s <= g.S; ++s) g.seg_start[s] = 5 * node_start[s];
    for (int s = 0; s < g.S; ++s) {
      const int64_t len = g.seg_start[s + 1] - g.seg_start[s];
      g.blk_start[s + 1] = g.blk_start[s] + std::max<int64_t>(1, (len + SEG_CH - 1) / SEG_CH);
    }
    g.B = (int)g.blk_start[g.S];
    g.block_seg.resize(g.B);
    for (int s = 0; s < g.S; ++s)
      for (int64_t b = g.blk_start[s]; b < g.blk_start[s + 1]; ++b) g.block_seg[b] = s;
    g.d_seg_start = dev_upload(g.seg_start);
    g.d_blk_start = dev_upload(g.blk_start);
    g.d_block_seg = dev_upload(g.block_seg);
    seg = g;
    dev_free(d_mask); dev_free(d_mask2); dev_free(d_svec); dev_free(flags);
    flags = dev_alloc<int>(g.S);
    d_mask = dev_alloc<uint8_t>(g.S);
    d_mask2 = dev_alloc<uint8_t>(g.S);
    d_svec = dev_alloc<double>(g.S);
    seg_act = g;
    seg_act.d_active = d_mask;
    seg_re = g;
    seg_re.d_active = d_mask2;
    dev_free(partials); dev_free(hdev); dev_free(ydev);
    partials = dev_alloc<double>((size_t)g.B * (KRYLOV_MAX + 2));
    hdev = dev_alloc<double>((size_t)g.S * HLD);
    ydev = dev_alloc<double>((size_t)g.S * HLD);
  }
  // per-segment 2-norms (scale: optional per-node weights)
  // (part, hv: reduction partials and result vector; null = the problem's own)
  // (g: the segments of x; null = the problem's unknown vector)
  std::vector<double> seg_norms(const double *x, hipStream_t st, const double *scale = nullptr,
                                double *part = nullptr, double *hv = nullptr, const SegHost *g = nullptr) {
    if (!part) part = partials;
    if (!hv) hv = hdev;
    const SegHost &sg = g ? *g : seg;
    launch_seg_norm2(sg, x, scale, part, st);
    launch_seg_reduce(sg, part, 1, hv, HLD, 0, st);
    std::vector<double> h((size_t)sg.S * HLD);
    download(h.data(), hv, sizeof(double) * h.size(), st);
    std::vector<double> out(sg.S);
    for (int s = 0; s < sg.S; ++s) out[s] = std::sqrt(h[(size_t)s * HLD]);
    return out;
  }
  // Small host->device uploads (masks, scalars, GMRES coefficients) go
  // through a pinned staging arena: each upload copies its bytes into a
  // fresh slice, so the source may change as soon as the call returns, and
  // a slice is reused only after a synchronisation of the stream(s) that
  // read it (when the arena is full or the stream changes).
  uint8_t *stage = nullptr;
  size_t stage_cap = 0, stage_off = 0;
  hipStream_t stage_st = nullptr;
  void upload(void *dst, const void *src, size_t bytes, hipStream_t st) {
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (stage_off > 0 && (st != stage_st || stage_off + need > stage_cap)) {
      HIPCHECK(hipStreamSynchronize(stage_st));
      stage_off = 0;
    }
    if (need > stage_cap) {
      if (stage) HIPCHECK(hipHostFree(stage));
      stage = nullptr;
      stage_cap = std::max<size_t>(need, (size_t)1 << 20);
      HIPCHECK(hipHostMalloc((void **)&stage, stage_cap, hipHostMallocDefault));
    }
    std::memcpy(stage + stage_off, src, bytes);
    HIPCHECK(hipMemcpyAsync(dst, stage + stage_off, bytes, hipMemcpyHostToDevice, st));
    stage_off += need;
    stage_st = st;
  }
  // Small device->host reads (Arnoldi coefficients, norms) land in a pinned
  // buffer and are copied out once the stream has synchronised (a pageable
  // destination makes each read a staged transfer).
  uint8_t *dl = nullptr;
  size_t dl_cap = 0;
  void download(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes > dl_cap) {  // no copy into dl is in flight: each read synchronises
      if (dl) HIPCHECK(hipHostFree(dl));
      dl = nullptr;
      dl_cap = std::max<size_t>(bytes, (size_t)1 << 16);
      HIPCHECK(hipHostMalloc((void **)&dl, dl_cap, hipHostMallocDefault));
    }
    HIPCHECK(hipMemcpyAsync(dl, src, bytes, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    std::memcpy(dst, dl, bytes);
  }
  // the staging arena and the download buffer, allocated up front so that
  // later transfers of up to their sizes never allocate
  void reserve_stage(size_t bytes) {
    if (!dl) {
      dl_cap = (size_t)1 << 16;
      HIPCHECK(hipHostMalloc((void **)&dl, dl_cap, hipHostMallocDefault));
    }
    if (stage) return;
    stage_cap = bytes;
    HIPCHECK(hipHostMalloc((void **)&stage, stage_cap, hipHostMallocDefault));
  }
  void upload_mask(uint8_t *d, const std::vector<uint8_t> &m, hipStream_t st) { upload(d, m.data(), m.size(), st); }
  void upload_scalars(const std::vector<double> &v, hipStream_t st) {
    upload(d_svec, v.data(), sizeof(double) * v.size(), st);
  }
  int64_t nvals() const { return 25 * mh.n + 10 * (int64_t)mh.col.size(); }
  const double *diag(const double *v) const { return v; }
  const double *off(const double *v) const { return v + 25 * mh.n; }

  double norm(const double *x, hipStream_t st, const double *scale = nullptr) {
    // the norm of the whole vector (all segments)
    const std::vector<double> v = seg_norms(x, st, scale);
    double t = 0.0;
    for (double e : v) t += e * e;
    return std::sqrt(t);
  }
  void ensure_krylov(int m) {
    if (kcap >= m) return;
    if (ws_base)
      fail(SEIRD_ERR_WORKSPACE, "GMRES restart " + std::to_string(m) + " above the " + std::to_string(ws_restart) +
                                    " reserved in the workspace");
    dev_free(V); dev_free(Zb);
    V = dev_alloc<double>((size_t)(m + 1) * N);
    Zb = dev_alloc<double>((size_t)m * N);
    kcap = m;
  }
};

// both packed triangular inverses of a coarse band with nt tile rows (tile 32)
// default super-block of the coarse inverses (tile rows): column chains of
// at most 128 rows at setup, against 2 ceil(nt / 128) block steps per solve
// (on the realistic coarse grid, 633 tile rows, 128 gives the shortest
// setup plus 16 solves per step; 64 and 32 shorten the setup a little and
// lengthen the solves more)
constexpr int COARSE_BLOCK = 128;
static inline double coarse_inverse_bytes(int64_t nt) { return 2.0 * (double)(nt * (nt + 1) / 2) * 1024 * 8; }
constexpr double COARSE_INVERSE_BUDGET = 16.0e9;

// Aggregation AMG V-cycle over dense 5x5 node blocks (the inner
// preconditioner of two-grid RAS-V3).  Level 0 is the coarse system in
// coarse positions; each level's nodes are grouped into aggregates that
// form the next level (piecewise-constant prolongation per component,
// Galerkin products as block sums); the last level is solved with an
// explicit dense inverse.
struct AmgLevel {
  int64_t n = 0, nslots = 0;
  int64_t *rowptr = nullptr;  // node graph without self loops (level 0: the coarse problem's)
  int32_t *col = nullptr;
  double *diag = nullptr, *off = nullptr;  // dense blocks: diag [n][25], off [nslots][25]
  double *dinv = nullptr;                  // inverted diagonal blocks
  double *x = nullptr, *b = nullptr, *r = nullptr;  // work vectors [5 n]
  // to the next level (all but the last)
  int64_t nagg = 0;
  int32_t *agg = nullptr;       // aggregate of each node
  int64_t *agg_ptr = nullptr;   // member nodes of each aggregate [nagg + 1]
  int32_t *agg_nodes = nullptr;
  int32_t *gdst = nullptr;      // next level's blocks: diagonal (-a-1) or slot
  int64_t *gptr = nullptr;      // sources of each next-level block [gnblk + 1]
  int32_t *gref = nullptr;      // source block: diagonal (-i-1) or slot of this level
  int64_t gnblk = 0;
  bool owns_graph = true;
};
struct AmgHier {
  std::vector<AmgLevel> lv;
  int nu = 1;
  double omega = 2.0 / 3.0;
  double *Ainv = nullptr;  // dense inverse of the last level (5 n_last)^2, row-major
  int m_last = 0;
  ~AmgHier() {
    for (AmgLevel &L : lv) {
      if (L.owns_graph) {
        dev_free(L.rowptr);
        dev_free(L.col);
        dev_free(L.diag);
        dev_free(L.off);
      }
      dev_free(L.dinv); dev_free(L.x); dev_free(L.b); dev_free(L.r);
      dev_free(L.agg); dev_free(L.agg_ptr); dev_free(L.agg_nodes);
      dev_free(L.gdst); dev_free(L.gptr); dev_free(L.gref);
    }
    dev_free(Ainv);
  }
};

// Two-grid RAS-V2 and V3 (Section 3.2): the coarse system solved by an
// inner GMRES preconditioned with one-level RAS on the coarse graph (V2)
// or with the aggregation AMG V-cycle (V3)
struct KrylovCoarse {
  seird_problem cp = nullptr;   // the coarse graph as a problem: vectors, Krylov basis, segment views
  seird_precond cpc = nullptr;  // V2: RAS on the coarse graph (dense off-diagonal blocks)
  AmgHier *amg = nullptr;       // V3: the AMG hierarchy
  double *cvals = nullptr;      // Galerkin coarse matrix: diag [nc][25], then off [slots][25]
  int32_t *gdst = nullptr;      // Galerkin block -> diagonal block or slot
  seird_krylov_opts ko{};
  int64_t solves = 0, its = 0, its_max = 0, unconverged = 0;
};
static void krylov_coarse_solve(seird_precond pc, const double *rc, double *xc, hipStream_t st);
static void krylov_coarse_free(KrylovCoarse *kc);
static void amg_setup(AmgHier &H, double *cdiag, double *coff, int *status, hipStream_t st);

struct seird_precond_s {
  seird_problem prob = nullptr;
  PrecondHost ph;
  bool dense_off = false;      // a coarse-graph RAS: dense off-diagonal node blocks (off [slots][25])
  KrylovCoarse *kc = nullptr;  // coarse_solver 2
  // coarse system prepared by the last setup: -1 none, 0 direct factors
  // (coarse_solver 0 or 1), 2 the Krylov coarse solver's matrix and RAS
  int coarse_prepared = -1;
  void *ws_base = nullptr;   // caller workspace holding its device arrays, if any
  int64_t nvec = 0;          // length of the vectors it applies to (bs * n_nodes)
  void *Fs = nullptr;        // subdomain factors as factorised (float64, or float32)
  bool sub_float = false;
  void *Fb = nullptr;        // bfloat16 copy for factor_prec 2, float32 copy for tile 16 + factor_prec 1
  double *Fc = nullptr;      // coarse factors (float64)
  SubInfo *subs_dev = nullptr;
  int32_t *order_dev = nullptr;
  ExtractEntry *ent_dev = nullptr;
  int32_t *ent_ptr = nullptr, *trow_ptr = nullptr, *trow_sub = nullptr;  // extraction entry and tile-row maps
  int32_t *l2g = nullptr;
  uint8_t *owned = nullptr;
  int32_t *env_row = nullptr, *env_lo = nullptr;  // subdomain row tables
  int *status = nullptr;
  int64_t *g2l_ptr = nullptr;
  int32_t *g2l_idx = nullptr;
  double *yloc = nullptr;
  int32_t *sub_seg = nullptr;  // instance of every subdomain (batches)
  std::vector<int32_t> sub_seg_host;
  int32_t *order_act = nullptr;  // batches: the active instances' subdomains, in LPT order
  std::vector<int32_t> order_act_host;
  int solve_threads = 256;     // workgroup size of the subdomain solves
  int max_nt = 0, max_bu = 0;
  // a setup made by a Newton step, kept for later steps (pc_keep_steps):
  // steps that reused it so far (-1: the last setup was not made by a step),
  // the step size it was made for, and GMRES iterations of its first solve
  int kept_steps = -1, kept_its = 0;
  double kept_dt = 0.0;
  // coarse
  SubInfo *coarse_dev = nullptr;
  int32_t *gp = nullptr, *gq = nullptr, *gref = nullptr, *cperm = nullptr;
  int64_t *gptr = nullptr;
  double *gw = nullptr;
  int64_t *z_ptr = nullptr, *zt_ptr = nullptr;
  int32_t *z_col = nullptr, *zt_col = nullptr;
  double *z_val = nullptr, *zt_val = nullptr;
  double *rc = nullptr, *xc = nullptr, *cscratch = nullptr, *ybuf = nullptr;
  double *cpart = nullptr;  // partial sums of the coarse triangular mat-vecs
  // explicit inverses of the coarse triangular factors (tile 32, when they
  // fit the budget); coarse_solver 1 uses them, 0 the band sweeps
  double *Xc = nullptr, *Wc = nullptr;
  int coarse_solver = 0;
  int coarse_block = 0;       // super-block of the inverses in Xc/Wc, in tile rows (as of the last setup)
  int coarse_block_next = 0;  // super-block the next setup forms them with
  double *t1 = nullptr;
  const double *vals_setup = nullptr;  // Jacobian of the last setup (borrowed)
  bool ready = false;
  // second stream (default priority) for the coarse factorisation, which
  // runs concurrently with the subdomain factorisation
  hipStream_t st_coarse = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // optional HIP-event timing of the subdomain solve launches
  bool timing = false;
  // captured Arnoldi-step graphs, keyed by what they bake in
  // (every setting that changes the launch sequence is part of the key)
  struct GraphKey {
    const void *prob, *V, *Zb, *vals;
    int j, transpose, masked;
    int coarse_solver, coarse_block, solve_threads;
    bool operator<(const GraphKey &o) const {
      return std::tie(prob, V, Zb, vals, j, transpose, masked, coarse_solver, coarse_block, solve_threads) <
             std::tie(o.prob, o.V, o.Zb, o.vals, o.j, o.transpose, o.masked, o.coarse_solver, o.coarse_block,
                      o.solve_threads);
    }
  };
  void clear_graphs() {
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  std::map<GraphKey, hipGraphExec_t> graphs;
  hipStream_t st_capture = nullptr;
  // replay the graph of `key`, capturing `launches` (on a private stream)
  // the first time
  template <class Fn>
  void run_graph(const GraphKey &key, Fn &&launches, hipStream_t st) {
    auto it = graphs.find(key);
    if (it == graphs.end()) {
      if (!st_capture) HIPCHECK(hipStreamCreateWithFlags(&st_capture, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      HIPCHECK(hipStreamBeginCapture(st_capture, hipStreamCaptureModeThreadLocal));
      try {
        launches(st_capture);
      } catch (...) {
        (void)hipStreamEndCapture(st_capture, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIPCHECK(hipStreamEndCapture(st_capture, &g));
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHECK(e);
      it = graphs.emplace(key, ex).first;
    }
    HIPCHECK(hipGraphLaunch(it->second, st));
  }
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t ev_used = 0;
  double ras_ms = 0.0;
  int ras_count = 0;
  // setup timing (when timing is on): extraction and subdomain factorisation
  hipEvent_t ev_set[3] = {nullptr, nullptr, nullptr};
  int set_count = 0;
  double set_extract_ms = 0.0, set_lu_ms = 0.0;

  double ras_bytes() const {
    // algorithmic bytes of one subdomain-solve launch: every stored factor
    // entry once, plus per local unknown the index, the owner flag and the
    // gathered value, plus the owned results written
    const int64_t nsubent = ph.factor_entries;
    const double fsz = ph.prec == 0 ? 8.0 : (ph.prec == 1 ? 4.0 : 2.0);
    return nsubent * fsz + (double)ph.l2g.size() * (4 + 1 + 8) + (double)nvec * 8;
  }
  // the same per instance of a batch (subdomains of that instance only)
  std::vector<double> seg_bytes;
  void set_instances(const std::vector<int32_t> &sub_seg_in, int n_inst) {
    sub_seg_host = sub_seg_in;
    sub_seg = dev_upload(sub_seg_host);
    order_act = dev_alloc<int32_t>(ph.n_sub);
    const double fsz = ph.prec == 0 ? 8.0 : (ph.prec == 1 ? 4.0 : 2.0);
    const int T = ph.tile;
    seg_bytes.assign(n_inst, 0.0);
    for (int i = 0; i < ph.n_sub; ++i) {
      const SubInfo &q = ph.subs[i];
      int64_t owned_n = 0;
      for (int l = 0; l < q.n_loc; ++l) owned_n += ph.owned[q.l2g_off + l];
      const int64_t tiles = q.env_off >= 0 ? ph.env_row[q.env_off + q.nt] : (int64_t)q.nt * (q.bl + q.bu + 1);
      seg_bytes[sub_seg_host[i]] += (double)tiles * T * T * fsz +
                                    (double)q.n_loc * (4 + 1 + 8) + (double)owned_n * 8;
    }
  }
  double ras_bytes_acc = 0.0;  // algorithmic bytes of the timed launches
  void harvest() {
    for (size_t k = 0; k < ev_used; ++k) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, ev[k].first, ev[k].second));
      ras_ms += t;
      ras_count++;
    }
    ev_used = 0;
  }

  ~seird_precond_s() {
    clear_graphs();
    krylov_coarse_free(kc);
    if (st_capture) (void)hipStreamDestroy(st_capture);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (st_coarse) (void)hipStreamDestroy(st_coarse);
    for (auto &e : ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    for (hipEvent_t e : ev_set)
      if (e) (void)hipEventDestroy(e);
    dev_free(Fs); dev_free(Fb); dev_free(Fc); dev_free(subs_dev); dev_free(order_dev); dev_free(ent_dev); dev_free(l2g);
    dev_free(env_row); dev_free(env_lo); dev_free(ent_ptr); dev_free(trow_ptr); dev_free(trow_sub);
    dev_free(owned); dev_free(status); dev_free(g2l_ptr); dev_free(g2l_idx); dev_free(yloc); dev_free(sub_seg);
    dev_free(order_act);
    dev_free(coarse_dev); dev_free(gp); dev_free(gq); dev_free(gref); dev_free(cperm); dev_free(gptr); dev_free(gw);
    dev_free(z_ptr); dev_free(zt_ptr); dev_free(z_col); dev_free(zt_col); dev_free(z_val); dev_free(zt_val);
    dev_free(rc); dev_free(xc); dev_free(cscratch); dev_free(ybuf); dev_free(t1); dev_free(Xc); dev_free(Wc);
    dev_free(cpart);
    if (ws_base) unregister_workspace(ws_base);
  }

  // factors read by the subdomain solves, in the storage precision ph.prec
  const void *factors() const {
    if (ph.prec == 0) return Fs;
    if (ph.prec == 1) return sub_float ? Fs : Fb;
    return Fb;
  }

  // seg_active / seg_active_host: device and host copies of the active
  // flags of a batch's instances (nullable)
  void ras(const double *r, double *z, int add, int transpose, hipStream_t st, const uint8_t *seg_active = nullptr,
           const std::vector<uint8_t> *seg_active_host = nullptr) {
    SolveLaunch sl;
    if (seg_active && sub_seg) {
      sl.sub_seg = sub_seg;
      sl.seg_active = seg_active;
    }
    sl.tile = ph.tile;
    sl.prec = ph.prec;
    sl.F = factors();
    sl.subs = subs_dev;
    sl.order = order_dev;
    sl.nblocks = ph.n_sub;
    if (sl.seg_active && seg_active_host && order_act) {
      // a batch with finished instances: launch only the active
      // instances' subdomains (compacted, still largest first), so that
      // the launch's time follows its bytes
      order_act_host.clear();
      for (int32_t idx : ph.order)
        if ((*seg_active_host)[sub_seg_host[idx]]) order_act_host.push_back(idx);
      if ((int)order_act_host.size() < ph.n_sub) {
        if (order_act_host.empty()) return;
        prob->upload(order_act, order_act_host.data(), sizeof(int32_t) * order_act_host.size(), st);
        sl.order = order_act;
        sl.nblocks = (int)order_act_host.size();
      }
    }
    sl.l2g = l2g;
    sl.owned = owned;
    sl.erow = env_row;
    sl.elo = env_lo;
    sl.r = r;
    sl.z = z;
    sl.add = add;
    sl.transpose = transpose;
    sl.yloc = yloc;
    sl.ybuf = ybuf;
    sl.threads = solve_threads;
    if (timing) {
      if (ev_used == ev.size()) {
        hipEvent_t a0, a1;
        HIPCHECK(hipEventCreate(&a0));
        HIPCHECK(hipEventCreate(&a1));
        ev.push_back({a0, a1});
      }
      HIPCHECK(hipEventRecord(ev[ev_used].first, st));
      launch_band_solve(sl, st);
      HIPCHECK(hipEventRecord(ev[ev_used].second, st));
      ev_used++;
      if (sl.seg_active && seg_active_host) {
        for (size_t k = 0; k < seg_bytes.size() && k < seg_active_host->size(); ++k)
          if ((*seg_active_host)[k]) ras_bytes_acc += seg_bytes[k];
      } else {
        ras_bytes_acc += ras_bytes();
      }
    } else {
      launch_band_solve(sl, st);
    }
    if (transpose) launch_gather_copies(g2l_ptr, g2l_idx, yloc, z, add, nvec, st);
  }

  // z += Z A_c^{-1} Z^T r  (or the transposed coarse operator)
  void coarse_add(const double *r, double *z, int transpose, hipStream_t st) {
    const bool krylov = coarse_solver >= 2;
    if ((krylov ? coarse_solver : 0) != coarse_prepared)
      fail(SEIRD_ERR_ARG, "coarse solver changed (direct, Krylov-RAS, Krylov-AMG) since the last setup");
    if (krylov && transpose) fail(SEIRD_ERR_ARG, "the Krylov coarse solvers have no transposed form");
    launch_coarse_restrict(zt_ptr, zt_col, zt_val, cperm, r, rc, ph.nc, st);
    if (krylov) {
      krylov_coarse_solve(this, rc, xc, st);
      launch_coarse_prolong(z_ptr, z_col, z_val, cperm, xc, z, prob->mh.n, st);
      return;
    }
    if (coarse_solver == 1) {
      launch_coarse_inverse_apply(Xc, Wc, Fc, ph.coarse, coarse_block, rc, xc, cscratch, cpart, transpose, st);
      launch_coarse_prolong(z_ptr, z_col, z_val, cperm, xc, z, prob->mh.n, st);
      return;
    }
    if (!transpose && ph.tile == 32 && ph.coarse.bl <= 16 && ph.coarse.bu <= 16) {
      launch_coarse_solve(Fc, coarse_dev, rc, xc, cscratch, st);
      launch_coarse_prolong(z_ptr, z_col, z_val, cperm, xc, z, prob->mh.n, st);
      return;
    }
    SolveLaunch sl;
    sl.tile = ph.tile;
    sl.prec = 0;  // the coarse factor is always float64
    sl.F = Fc;
    sl.subs = coarse_dev;
    sl.order = nullptr;
    sl.nblocks = 1;
    sl.wide = true;
    sl.r = rc;
    sl.z = xc;
    sl.transpose = transpose;
    sl.ybuf = cscratch;
    launch_band_solve(sl, st);
    launch_coarse_prolong(z_ptr, z_col, z_val, cperm, xc, z, prob->mh.n, st);
  }

  // seg_active (device, nullable): active flag per instance of a batch;
  // the subdomain solves of inactive instances are skipped (one-level only)
  void apply(const double *vals, const double *r, double *z, int transpose, hipStream_t st,
             const uint8_t *seg_active = nullptr, const std::vector<uint8_t> *seg_active_host = nullptr) {
    if (!ready) fail(SEIRD_ERR_ARG, "preconditioner used before setup");
    seird_problem P = prob;
    if (!ph.two_level) {
      ras(r, z, 0, transpose, st, seg_active, seg_active_host);
      return;
    }
    // multiplicative two-grid: pre-smooth, coarse correction, post-smooth
    ras(r, z, 0, transpose, st);                                               // z1 = M r
    launch_spmv(P->md, P->diag(vals), P->off(vals), z, r, t1, transpose, st);  // r1 = r - A z1
    coarse_add(t1, z, transpose, st);                                          // z2 = z1 + Q r1
    launch_spmv(P->md, P->diag(vals), P->off(vals), z, r, t1, transpose, st);  // r2 = r - A z2
    ras(t1, z, 1, transpose, st);                                              // z = z2 + M r2
  }
};

// ------------------------------------------------------------------------
// GMRES (right preconditioned, restarted, CGS + one conditional DGKS pass),
// run independently on every active segment (instance): per-segment
// Hessenberg, Givens rotations, stopping and restarts; the segments still
// running advance in lockstep through shared kernel launches that mask the
// others.  A single problem is one segment.
// ------------------------------------------------------------------------
// Device work of one GMRES run: the Krylov basis V [m+1][N], the
// preconditioned vectors Z [m][N], the reduction partials and the small
// coefficient vector.  Null members are taken from the problem (its basis
// allocated on first use).
struct KrylovWork {
  double *V = nullptr, *Zb = nullptr, *partials = nullptr, *hdev = nullptr;
};

// The linear system GMRES runs on: vector length, the segments of its
// vectors (plain, active-masked, second mask), y = A x or y = b - A x, and
// z = M^{-1} r (null: no preconditioner; masks for a batch's instances).
// Graph capture of the Arnoldi steps is available only through `pc`.
struct GmresOps {
  int64_t N = 0;
  const SegHost *seg = nullptr, *seg_act = nullptr, *seg_re = nullptr;
  std::function<void(const double *x, const double *b, double *y, hipStream_t)> spmv;
  std::function<void(const double *r, double *z, hipStream_t, const uint8_t *, const std::vector<uint8_t> *)> prec;
  seird_precond pc = nullptr;  // for graph capture (coupled systems only)
  const double *vals = nullptr;
  int transpose = 0;
};

// a double for messages, in %g form
static std::string fmt_g(double v) {
  char b[32];
  std::snprintf(b, sizeof b, "%.3g", v);
  return b;
}

static void gmres_core(seird_problem P, const GmresOps &ops, const double *b, double *x, const seird_krylov_opts &o,
                       std::vector<seird_krylov_stats> &stats, const std::vector<uint8_t> &active_in, hipStream_t st,
                       const KrylovWork &work);

static void gmres_impl(seird_problem P, seird_precond pc, const double *vals, const double *b, double *x,
                       const seird_krylov_opts &o, std::vector<seird_krylov_stats> &stats,
                       const std::vector<uint8_t> &active_in, int transpose, hipStream_t st,
                       const KrylovWork &work = KrylovWork{}) {
  GmresOps ops;
  ops.N = P->N;
  ops.seg = &P->seg;
  ops.seg_act = &P->seg_act;
  ops.seg_re = &P->seg_re;
  ops.spmv = [P, vals, transpose](const double *xx, const double *bb, double *y, hipStream_t s) {
    launch_spmv(P->md, P->diag(vals), P->off(vals), xx, bb, y, transpose, s);
  };
  if (pc)
    ops.prec = [pc, vals, transpose](const double *r, double *z, hipStream_t s, const uint8_t *dm,
                                     const std::vector<uint8_t> *hm) { pc->apply(vals, r, z, transpose, s, dm, hm); };
  ops.pc = pc;
  ops.vals = vals;
  ops.transpose = transpose;
  gmres_core(P, ops, b, x, o, stats, active_in, st, work);
}

static void gmres_core(seird_problem P, const GmresOps &ops, const double *b, double *x, const seird_krylov_opts &o,
                       std::vector<seird_krylov_stats> &stats, const std::vector<uint8_t> &active_in, hipStream_t st,
                       const KrylovWork &work) {
  const int64_t N = ops.N;
  const SegHost &seg = *ops.seg, &seg_act = *ops.seg_act, &seg_re = *ops.seg_re;
  const seird_precond pc = ops.pc;
  const double *vals = ops.vals;
  const int transpose = ops.transpose;
  const int S = seg.S;
  const int HLD = P->HLD;
  const int m = o.restart;
  if (m < 1 || m > KRYLOV_MAX - 1) fail(SEIRD_ERR_ARG, "restart must be in [1, 31]");
  if (o.max_it < 0) fail(SEIRD_ERR_ARG, "max_it must be >= 0");
  if (!work.V) P->ensure_krylov(m);
  double *V = work.V ? work.V : P->V, *Zb = work.Zb ? work.Zb : P->Zb;
  double *const partials = work.partials ? work.partials : P->partials;
  double *const hdev = work.hdev ? work.hdev : P->hdev;
  stats.assign(S, seird_krylov_stats{});
  launch_fill(x, 0.0, N, st);
  const std::vector<double> bnorm = P->seg_norms(b, st, nullptr, partials, hdev, &seg);
  std::vector<uint8_t> act(S, 0);
  std::vector<double> target(S, 0.0), beta(S, 0.0), sc(S, 0.0);
  std::vector<int> its(S, 0);
  for (int s = 0; s < S; ++s) {
    stats[s].bnorm = stats[s].resid = bnorm[s];
    if (!active_in[s]) continue;
    if (!std::isfinite(bnorm[s])) fail(SEIRD_ERR_NONFINITE, "nonfinite right-hand side");
    target[s] = std::max(o.rtol * bnorm[s], o.atol);
    if (bnorm[s] <= target[s]) {
      stats[s].reason = 1;
      continue;
    }
    act[s] = 1;
    beta[s] = bnorm[s];
    sc[s] = 1.0 / beta[s];
  }
  auto any = [](const std::vector<uint8_t> &v) {
    for (uint8_t e : v)
      if (e) return true;
    return false;
  };
  if (!any(act)) return;
  P->upload_mask(P->d_mask, act, st);
  P->upload_scalars(sc, st);
  launch_seg_axpby(seg_act, V, b, P->d_svec, 0.0, st);
  std::vector<double> H((size_t)S * (m + 1) * m), cs((size_t)S * m), sn((size_t)S * m), g((size_t)S * (m + 1));
  std::vector<double> hbuf((size_t)S * HLD), ybuf((size_t)S * HLD);
  const double eta = 1.0 / std::sqrt(2.0);
  auto Hs = [&](int s, int i, int j) -> double & { return H[(size_t)s * (m + 1) * m + (size_t)i * m + j]; };
  // x += Z y for the segments in `fin`, each with k columns
  auto update = [&](const std::vector<uint8_t> &fin, int k) {
    for (int s = 0; s < S; ++s) {
      if (!fin[s]) continue;
      double *y = &ybuf[(size_t)s * HLD];
      for (int i = k - 1; i >= 0; --i) {
        double t = g[(size_t)s * (m + 1) + i];
        for (int l = i + 1; l < k; ++l) t -= Hs(s, i, l) * y[l];
        y[i] = t / Hs(s, i, i);
      }
    }
    P->upload(P->ydev, ybuf.data(), sizeof(double) * ybuf.size(), st);
    P->upload_mask(P->d_mask2, fin, st);
    launch_seg_gemv_update(seg_re, x, Zb, N, P->ydev, HLD, k, st);
  };
  while (any(act)) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    for (int s = 0; s < S; ++s)
      if (act[s]) g[(size_t)s * (m + 1)] = beta[s];
    std::vector<uint8_t> cyc = act;  // segments running in this cycle
    int j = 0;
    for (; j < m && any(cyc); ++j) {
      double *vj = V + (int64_t)j * N, *zj = Zb + (int64_t)j * N, *w = V + (int64_t)(j + 1) * N;
      // (a single segment's mask is set before the cycle and cannot change
      // within it: the cycle ends when its one segment finishes)
      if (S > 1) P->upload_mask(P->d_mask, cyc, st);
      // z_j = M^{-1} v_j, w = A z_j, then h = V^T w, w -= V h, |w|^2
      auto step_launches = [&](hipStream_t s) {
        if (ops.prec)
          ops.prec(vj, zj, s, S > 1 ? P->d_mask : nullptr, S > 1 ? &cyc : nullptr);
        else
          HIPCHECK(hipMemcpyAsync(zj, vj, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        ops.spmv(zj, nullptr, w, s);
        launch_seg_mdot(seg_act, V, N, j + 1, w, 1, partials, s);
        launch_seg_reduce(seg, partials, j + 2, hdev, HLD, 0, s);
        launch_seg_maxpy_norm(seg_act, w, V, N, hdev, HLD, j + 1, partials, s);
        launch_seg_reduce(seg, partials, 1, hdev, HLD, j + 2, s);
      };
      // (graphs only for a single instance: a batch's launches depend on
      // which instances are still running)
      if (pc && o.graphs && !pc->timing && S == 1 && pc->coarse_solver < 2)
        pc->run_graph({P, V, Zb, vals, j, transpose, S > 1, pc->coarse_solver, pc->coarse_block, pc->solve_threads},
                      step_launches, st);
      else
        step_launches(st);
      P->download(hbuf.data(), hdev, sizeof(double) * hbuf.size(), st);
      std::vector<uint8_t> re(S, 0);
      std::vector<double> wn(S, 0.0);
      bool any_re = false;
      for (int s = 0; s < S; ++s) {
        if (!cyc[s]) continue;
        for (int i = 0; i <= j; ++i) Hs(s, i, j) = hbuf[(size_t)s * HLD + i];
        const double wn0 = std::sqrt(hbuf[(size_t)s * HLD + j + 1]);
        wn[s] = std::sqrt(hbuf[(size_t)s * HLD + j + 2]);
        if (!std::isfinite(wn[s]) || !std::isfinite(wn0)) fail(SEIRD_ERR_NONFINITE, "nonfinite Arnoldi vector");
        if (wn[s] < eta * wn0) {
          re[s] = 1;
          any_re = true;
        }
      }
      if (any_re) {  // DGKS: one reorthogonalisation pass for those segments
        P->upload_mask(P->d_mask2, re, st);
        launch_seg_mdot(seg_re, V, N, j + 1, w, 0, partials, st);
        launch_seg_reduce(seg, partials, j + 1, hdev, HLD, 0, st);
        launch_seg_maxpy_norm(seg_re, w, V, N, hdev, HLD, j + 1, partials, st);
        launch_seg_reduce(seg, partials, 1, hdev, HLD, j + 1, st);
        P->download(hbuf.data(), hdev, sizeof(double) * hbuf.size(), st);
        for (int s = 0; s < S; ++s) {
          if (!re[s]) continue;
          for (int i = 0; i <= j; ++i) Hs(s, i, j) += hbuf[(size_t)s * HLD + i];
          wn[s] = std::sqrt(hbuf[(size_t)s * HLD + j + 1]);
        }
      }
      for (int s = 0; s < S; ++s) sc[s] = (cyc[s] && wn[s] > 0.0) ? 1.0 / wn[s] : 0.0;
      if (S == 1) {  // the scale as a kernel argument: no upload
        launch_axpby(w, w, sc[0], nullptr, 0, 0.0, N, reduction_blocks(N), st);
      } else {
        P->upload_scalars(sc, st);
        launch_seg_axpby(seg_act, w, w, P->d_svec, 0.0, st);
      }
      std::vector<uint8_t> fin(S, 0);
      std::vector<int> kfin(S, 0);
      bool any_fin = false;
      for (int s = 0; s < S; ++s) {
        if (!cyc[s]) continue;
        Hs(s, j + 1, j) = wn[s];
        double *c = &cs[(size_t)s * m], *sn_ = &sn[(size_t)s * m], *gg = &g[(size_t)s * (m + 1)];
        for (int i = 0; i < j; ++i) {
          const double t = c[i] * Hs(s, i, j) + sn_[i] * Hs(s, i + 1, j);
          Hs(s, i + 1, j) = -sn_[i] * Hs(s, i, j) + c[i] * Hs(s, i + 1, j);
          Hs(s, i, j) = t;
        }
        const double den = std::hypot(Hs(s, j, j), Hs(s, j + 1, j));
        int reason = 0;
        if (den == 0.0) {
          reason = 2;  // exact breakdown: the first j columns hold the solution
          kfin[s] = j;
        } else {
          c[j] = Hs(s, j, j) / den;
          sn_[j] = Hs(s, j + 1, j) / den;
          Hs(s, j, j) = den;
          Hs(s, j + 1, j) = 0.0;
          gg[j + 1] = -sn_[j] * gg[j];
          gg[j] = c[j] * gg[j];
          ++its[s];
          kfin[s] = j + 1;
          const double res = std::fabs(gg[j + 1]);
          stats[s].resid = res;
          if (res < target[s]) reason = 1;
          else if (res > o.dtol * bnorm[s]) reason = SEIRD_ERR_DIVERGED;
          else if (its[s] >= o.max_it) reason = SEIRD_ERR_NOT_CONVERGED;
          else if (wn[s] == 0.0) reason = 2;
        }
        if (reason != 0) {
          stats[s].reason = reason;
          stats[s].its = its[s];
          fin[s] = 1;
          any_fin = true;
        }
      }
      if (any_fin) {
        for (int kk : {j + 1, j}) {
          std::vector<uint8_t> f(S, 0);
          bool anyf = false;
          for (int s = 0; s < S; ++s)
            if (fin[s] && kfin[s] == kk) {
              f[s] = 1;
              anyf = true;
            }
          if (anyf && kk > 0) update(f, kk);
        }
        for (int s = 0; s < S; ++s)
          if (fin[s]) {
            cyc[s] = 0;
            act[s] = 0;
          }
      }
    }
    // segments that completed a full cycle: update, restart from the true residual
    if (any(cyc)) {
      update(cyc, m);
      P->upload_mask(P->d_mask, cyc, st);
      ops.spmv(x, b, V, st);
      const std::vector<double> bt = P->seg_norms(V, st, nullptr, partials, hdev, &seg);
      for (int s = 0; s < S; ++s) {
        if (!cyc[s]) continue;
        beta[s] = bt[s];
        stats[s].resid = bt[s];
        if (bt[s] <= target[s]) {
          stats[s].reason = 1;
          stats[s].its = its[s];
          act[s] = 0;
          cyc[s] = 0;
        }
        sc[s] = cyc[s] ? 1.0 / bt[s] : 0.0;
      }
      if (any(cyc)) {
        P->upload_mask(P->d_mask, cyc, st);
        P->upload_scalars(sc, st);
        launch_seg_axpby(seg_act, V, V, P->d_svec, 0.0, st);
      }
    }
  }
  HIPCHECK(hipStreamSynchronize(st));
}

static void precond_setup_impl(seird_precond pc, const double *vals, hipStream_t st);

// One implicit step on every segment (instance) of u: each segment runs its
// own Newton iteration (own residual scale, stopping test and counters); a
// converged segment is frozen while the others continue.  The
// preconditioner is shared: its setup schedule (first iteration, then every
// pc_reuse + 1 iterations, or when a reused setup failed or stopped paying)
// applies to all segments together.
static void step_impl(seird_problem p, seird_precond pc, double *u, double dt, const double *src,
                      const seird_newton_opts *nopts, const seird_krylov_opts *kopts,
                      std::vector<seird_step_stats> &stats, hipStream_t st, double t_next) {
  const ParamsDev Pt = p ? p->params_at(t_next) : ParamsDev{};  // coefficients at the end of the step
  if (!p || !u || !nopts || !kopts) fail(SEIRD_ERR_ARG, "null argument");
  if (nopts->max_it < 0 || nopts->max_it > SEIRD_MAX_NEWTON) fail(SEIRD_ERR_ARG, "Newton max_it out of range");
  if (nopts->pc_reuse < 0) fail(SEIRD_ERR_ARG, "pc_reuse must be >= 0");
  if (nopts->pc_keep_steps < 0) fail(SEIRD_ERR_ARG, "pc_keep_steps must be >= 0");
  using clk = std::chrono::steady_clock;
  auto ms = [](clk::time_point a0, clk::time_point b0) {
    return std::chrono::duration<double, std::milli>(b0 - a0).count();
  };
  const int S = p->seg.S;
  stats.assign(S, seird_step_stats{});
  const int64_t N = p->N;
  HIPCHECK(hipMemcpyAsync(p->u_prev, u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  // per-instance state flags: bit 0 a nonfinite entry, bit 1 N <= 0 at a node
  auto state_flags = [&](const double *x) {
    HIPCHECK(hipMemsetAsync(p->flags, 0, sizeof(int) * S, st));
    launch_check_state(x, p->mh.n, p->md.inst, p->flags, st);
    std::vector<int> f(S, 0);
    HIPCHECK(hipMemcpyAsync(f.data(), p->flags, sizeof(int) * S, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    return f;
  };
  auto where = [&](int s) { return S > 1 ? " in instance " + std::to_string(s) : std::string(); };
  {
    const std::vector<int> f = state_flags(u);
    for (int s = 0; s < S; ++s) {
      if (f[s] & 1) fail(SEIRD_ERR_NONFINITE, "nonfinite state" + where(s));
      if (f[s] & 2) fail(SEIRD_ERR_STATE, "total density N <= 0 at a node" + where(s));
    }
  }
  const std::vector<double> scale = p->seg_norms(p->u_prev, st, p->md.mass);
  const std::vector<double> unorm = p->seg_norms(p->u_prev, st);
  double *diag = p->vals, *off = p->vals + 25 * p->mh.n;
  std::vector<uint8_t> act(S, 1);
  int last_setup = 0, its_fresh = 0;
  bool stale = false;
  std::vector<seird_krylov_stats> ks;
  double t_res = 0, t_jac = 0, t_set = 0, t_gm = 0;
  int setups = 0;
  for (int k = 0;; ++k) {
    auto t0 = clk::now();
    launch_residual(p->md, Pt, p->gfield, u, p->u_prev, dt, src, p->F, st);
    const std::vector<double> fn = p->seg_norms(p->F, st);
    t_res += ms(t0, clk::now());
    bool any_act = false;
    for (int s = 0; s < S; ++s) {
      if (!act[s]) continue;
      stats[s].res_hist[k] = fn[s] / scale[s];
      if (!std::isfinite(fn[s])) fail(SEIRD_ERR_NONFINITE, "nonfinite residual");
      if (fn[s] <= nopts->tol * scale[s])
        act[s] = 0;
      else
        any_act = true;
    }
    if (!any_act) break;
    if (k >= nopts->max_it) {
      std::string msg = "Newton did not converge in " + std::to_string(nopts->max_it) + " iterations";
      for (int s = 0; s < S; ++s) {
        if (!act[s]) continue;
        msg += where(s) + " (scaled residuals";
        for (int i = std::max(0, k - 4); i <= k; ++i) msg += " " + std::to_string(stats[s].res_hist[i]);
        msg += ", tolerance " + std::to_string(nopts->tol) + ")";
        break;
      }
      fail(SEIRD_ERR_NOT_CONVERGED, msg);
    }
    t0 = clk::now();
    launch_jacobian(p->md, Pt, p->gfield, u, dt, diag, off, st);
    HIPCHECK(hipStreamSynchronize(st));
    t_jac += ms(t0, clk::now());
    t0 = clk::now();
    bool fresh = false;
    // the first iteration may take a setup kept from an earlier step
    const bool keep = k == 0 && pc && nopts->pc_keep_steps > 0 && pc->prob == p && pc->kept_steps >= 0 &&
                      pc->kept_steps < nopts->pc_keep_steps && pc->kept_dt == dt;
    if (keep) {
      ++pc->kept_steps;
      its_fresh = pc->kept_its;
    } else if (pc && (k == 0 || stale || (k - last_setup) > nopts->pc_reuse)) {
      precond_setup_impl(pc, p->vals, st);
      ++setups;
      last_setup = k;
      stale = false;
      fresh = true;
    }
    t_set += ms(t0, clk::now());
    t0 = clk::now();
    launch_axpby(p->rhs, p->F, -1.0, nullptr, 0, 0.0, N, reduction_blocks(N), st);
    // A reused setup gets an iteration budget of twice the last fresh count
    // plus 5 (at least 10): beyond it the setup counts as failed and is
    // rebuilt, instead of letting a stale preconditioner run to max_it.
    seird_krylov_opts ko = *kopts;
    if (pc && !fresh && its_fresh > 0) ko.max_it = std::min(kopts->max_it, std::max(10, 2 * its_fresh + 5));
    gmres_impl(p, pc, p->vals, p->rhs, p->delta, ko, ks, act, 0, st);
    bool failed = false;
    for (int s = 0; s < S; ++s)
      if (act[s] && ks[s].reason < 0) failed = true;
    std::vector<int> its_first(S, 0);
    if (pc && !fresh && failed) {
      // a reused setup failed: rebuild it from the current Jacobian and retry
      auto t1 = clk::now();
      precond_setup_impl(pc, p->vals, st);
      ++setups;
      last_setup = k;
      t_set += ms(t1, clk::now());
      for (int s = 0; s < S; ++s) its_first[s] = ks[s].its;
      gmres_impl(p, pc, p->vals, p->rhs, p->delta, *kopts, ks, act, 0, st);
      fresh = true;
    }
    int its_max = 0;
    for (int s = 0; s < S; ++s)
      if (act[s]) its_max = std::max(its_max, ks[s].its + its_first[s]);
    if (fresh) {
      its_fresh = its_max;
      // this step's own setup: a later step may keep it
      pc->kept_steps = 0;
      pc->kept_dt = dt;
      pc->kept_its = its_max;
    } else if (its_max > 2 * its_fresh + 5) {
      stale = true;  // reuse no longer pays
    }
    t_gm += ms(t0, clk::now());
    if (pc && pc->timing) {
      HIPCHECK(hipStreamSynchronize(st));
      pc->harvest();
    }
    for (int s = 0; s < S; ++s) {
      if (!act[s]) continue;
      stats[s].gmres_its[k] = ks[s].its + its_first[s];
      stats[s].gmres_its_total += ks[s].its + its_first[s];
      stats[s].newton_its = k + 1;
      if (ks[s].reason == SEIRD_ERR_DIVERGED) fail(SEIRD_ERR_DIVERGED, "GMRES diverged" + where(s));
      if (ks[s].reason == SEIRD_ERR_NOT_CONVERGED) {
        ++stats[s].inexact_solves;
        if (nopts->strict_linear)
          fail(SEIRD_ERR_NOT_CONVERGED, "GMRES reached max_it (" + std::to_string(ks[s].its + its_first[s]) +
                                            " iterations, residual " + std::to_string(ks[s].resid) + " of " +
                                            std::to_string(ks[s].bnorm) + ") in Newton iteration " +
                                            std::to_string(k + 1) + where(s));
      }
    }
    // max_it without convergence (strict_linear = 0): the inexact Newton
    // update is still taken and counted in inexact_solves; frozen segments
    // have a zero update
    launch_axpby(u, p->delta, 1.0, nullptr, 0, 1.0, N, reduction_blocks(N), st);
    // Positivity safeguard: an instance whose new iterate has N <= 0 at a
    // node gets its update halved (u -= delta / 2, delta /= 2), at most
    // MAX_HALVINGS times.  The root is unchanged; only the path to it.
    constexpr int MAX_HALVINGS = 10;
    for (int bt = 0;; ++bt) {
      const std::vector<int> f = state_flags(u);
      std::vector<uint8_t> bad(S, 0);
      bool any_bad = false;
      for (int s = 0; s < S; ++s) {
        auto diag_msg = [&]() {
          std::string h;
          for (int i = 0; i <= k; ++i) h += (i ? ", " : "") + std::to_string(stats[s].res_hist[i]);
          return where(s) + " after Newton iteration " + std::to_string(k + 1) + " (GMRES its " +
                 std::to_string(ks[s].its) + ", reason " + std::to_string(ks[s].reason) + "; scaled residuals " +
                 h + ")";
        };
        if (f[s] & 1) fail(SEIRD_ERR_NONFINITE, "nonfinite state" + diag_msg());
        if (f[s] & 2) {
          if (bt == MAX_HALVINGS)
            fail(SEIRD_ERR_STATE, "total density N <= 0 at a node" + diag_msg() + " after " +
                                      std::to_string(MAX_HALVINGS) + " halvings");
          bad[s] = 1;
          any_bad = true;
          ++stats[s].backtracks;
        }
      }
      if (!any_bad) break;
      p->upload_mask(p->d_mask2, bad, st);
      p->upload_scalars(std::vector<double>(S, -0.5), st);
      launch_seg_axpby(p->seg_re, u, p->delta, p->d_svec, 1.0, st);
      p->upload_scalars(std::vector<double>(S, 0.5), st);
      launch_seg_axpby(p->seg_re, p->delta, p->delta, p->d_svec, 0.0, st);
    }
    const std::vector<double> dn = p->seg_norms(p->delta, st);
    for (int s = 0; s < S; ++s)
      if (act[s]) stats[s].eps = dn[s] / unorm[s];
  }
  for (int s = 0; s < S; ++s) {
    stats[s].pc_setups = setups;
    stats[s].t_residual_ms = t_res;
    stats[s].t_jacobian_ms = t_jac;
    stats[s].t_setup_ms = t_set;
    stats[s].t_gmres_ms = t_gm;
  }
  if (pc && pc->timing) {
    for (int s = 0; s < S; ++s) {
      stats[s].t_ras_kernel_ms = pc->ras_ms;
      stats[s].n_ras_launches = pc->ras_count;
      stats[s].ras_bytes_per_launch = pc->ras_count ? pc->ras_bytes_acc / pc->ras_count : pc->ras_bytes();
    }
    pc->ras_ms = 0.0;
    pc->ras_count = 0;
    pc->ras_bytes_acc = 0.0;
  }
}

extern "C" {

const char *seird_last_error(void) { return g_last_error.c_str(); }

seird_status seird_device_allocations(int64_t *count, int64_t *bytes) {
  API_BEGIN
  if (count) *count = g_dev_allocs.load();
  if (bytes) *bytes = g_dev_alloc_bytes.load();
  API_END
}
const char *seird_version(void) { return "libseird 0.1 gfx950"; }

struct seird_mesh_s {
  MeshHost mh;
};

// A problem on a built mesh (the host data are copied).  Device memory
// comes from the active arena, if any (see Arena).
static seird_problem problem_create_impl(const MeshHost &mh, const seird_params &params) {
  auto P = new seird_problem_s();
  try {
    if (!measuring()) {
      HIPCHECK(hipGetDevice(&P->device));
      int lds = 0;
      if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) == hipSuccess && lds > 0)
        P->lds_limit = (size_t)lds;
      int cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && cus > 0)
        P->n_cu = cus;
    }
    P->mh = mh;
    P->P = to_dev(params);
    const MeshHost &m = P->mh;
    P->md.n = m.n;
    P->md.nslots = (int64_t)m.col.size();
    P->md.rowptr = dev_upload(m.rowptr);
    P->md.col = dev_upload(m.col);
    P->md.tslot = dev_upload(m.tslot);
    P->md.mass = dev_upload(m.mass);
    P->md.inc_ptr = dev_upload(m.inc_ptr);
    P->md.inc_j = dev_upload(m.inc_j);
    P->md.inc_l = dev_upload(m.inc_l);
    P->md.inc_sj = dev_upload(m.inc_sj);
    P->md.slot_row = dev_upload(m.slot_row);
    P->md.slot_ek = dev_upload(m.slot_ek);
    P->md.kd = dev_upload(m.kd);
    P->md.ko = dev_upload(m.ko);
    P->md.kw = dev_upload(m.kw);
    P->md.inc_sl = dev_upload(m.inc_sl);
    P->md.inc_K = dev_upload(m.inc_K);
    P->d_cmass_d = dev_upload(m.cmass_d);
    P->d_cmass_o = dev_upload(m.cmass_o);
    P->d_bnd_ptr = dev_upload(m.bnd_ptr);
    P->d_bnd_j = dev_upload(m.bnd_j);
    P->d_bnd_nl = dev_upload(m.bnd_nl);
    P->d_qflux = dev_alloc<double>((size_t)10 * m.n);
    P->md.bnd_ptr = P->d_bnd_ptr;
    P->md.bnd_j = P->d_bnd_j;
    P->md.bnd_nl = P->d_bnd_nl;
    P->N = 5 * m.n;
    P->nb = reduction_blocks(P->N);
    P->setup_segments({0, m.n});
    P->u_prev = dev_alloc<double>(P->N);
    P->F = dev_alloc<double>(P->N);
    P->rhs = dev_alloc<double>(P->N);
    P->delta = dev_alloc<double>(P->N);
    P->w1 = dev_alloc<double>(P->N);
    P->vals = dev_alloc<double>(P->nvals());
    if (!measuring()) {
      P->reserve_stage((size_t)1 << 20);
      (void)static_scratch();  // this device's scratch address, looked up once
    }
  } catch (...) {
    delete P;
    throw;
  }
  return P;
}

seird_status seird_problem_create(int64_t n_nodes, const double *xy, int64_t n_tri, const int32_t *tri,
                                  const seird_params *params, seird_problem *out) {
  API_BEGIN
  if (!out || !params) fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  MeshHost mh;
  build_mesh(n_nodes, xy, n_tri, tri, mh);
  *out = problem_create_impl(mh, *params);
  API_END
}

seird_status seird_mesh_create(int64_t n_nodes, const double *xy, int64_t n_tri, const int32_t *tri,
                               seird_mesh *out) {
  API_BEGIN
  if (!out) fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  auto m = new seird_mesh_s();
  try {
    build_mesh(n_nodes, xy, n_tri, tri, m->mh);
  } catch (...) {
    delete m;
    throw;
  }
  *out = m;
  API_END
}

void seird_mesh_destroy(seird_mesh m) { delete m; }

seird_status seird_mesh_info(seird_mesh m, int64_t *n_nodes, int64_t *n_slots) {
  API_BEGIN
  if (!m) fail(SEIRD_ERR_ARG, "null mesh");
  if (n_nodes) *n_nodes = m->mh.n;
  if (n_slots) *n_slots = (int64_t)m->mh.col.size();
  API_END
}

seird_status seird_problem_create_from_mesh(seird_mesh m, const seird_params *params, seird_problem *out) {
  API_BEGIN
  if (!m || !params || !out) fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  *out = problem_create_impl(m->mh, *params);
  API_END
}

static seird_precond precond_create_impl(seird_problem p, const seird_schwarz_opts *opts, const int32_t *part,
                                         int bs, const PrecondHost *proto = nullptr);

// bytes of the adjoint-record pool of a workspace
static size_t tape_pool_bytes(int64_t n, const seird_workspace_opts &wo) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  if (wo.tape_states <= 0) return 0;
  return (size_t)wo.tape_states * up(sizeof(double) * 5 * (size_t)n) + 2 * up(sizeof(int32_t) * (size_t)n) +
         up(sizeof(int64_t) * ((size_t)std::max(wo.n_regions_max, 0) + 1)) +
         up(sizeof(double) * (5 * (size_t)((n + 255) / 256) + 8)) + 4096;
}

// The problem (and, with opts, its preconditioner) with every device array
// taken from `arena`; in measure mode nothing is allocated.
static void create_in_arena(const MeshHost &mh, const seird_params &params, const seird_schwarz_opts *opts,
                            const int32_t *part, const seird_workspace_opts &wo, Arena &arena, seird_problem *prob,
                            seird_precond *pc) {
  if (wo.restart_max < 1 || wo.restart_max > KRYLOV_MAX - 1) fail(SEIRD_ERR_ARG, "restart_max must be in [1, 31]");
  if (wo.tape_states < 0 || wo.n_regions_max < 0) fail(SEIRD_ERR_ARG, "negative workspace reservation");
  ArenaScope scope(&arena);
  seird_problem P = problem_create_impl(mh, params);
  try {
    P->ensure_krylov(wo.restart_max);
    P->gfield_store = dev_alloc<double>(mh.n);
    if (wo.csr_pattern) {
      const int64_t nnz = 25 * ((int64_t)mh.col.size() + mh.n);
      P->csr_rowptr = dev_alloc<int64_t>(5 * mh.n + 1);
      P->csr_col = dev_alloc<int32_t>(nnz);
      P->csr_reserved = true;
    }
    const size_t tb = tape_pool_bytes(mh.n, wo);
    if (tb > 0) {
      P->tape_pool.base = static_cast<uint8_t *>(dev_alloc_bytes(tb));
      P->tape_pool.cap = tb;
    }
    if (opts) *pc = precond_create_impl(P, opts, part, NC);
  } catch (...) {
    delete P;
    throw;
  }
  *prob = P;
}

seird_status seird_workspace_bytes(seird_mesh m, const seird_schwarz_opts *opts, const int32_t *part,
                                   const seird_workspace_opts *wo, int64_t *bytes) {
  API_BEGIN
  if (!m || !wo || !bytes) fail(SEIRD_ERR_ARG, "null argument");
  if (opts && !part) fail(SEIRD_ERR_ARG, "a preconditioner needs the partition");
  // run the creation with a measuring arena: the same allocations in the
  // same order, sizes only (the fake addresses are never dereferenced)
  Arena a;
  a.measure = true;
  a.base = reinterpret_cast<uint8_t *>((uintptr_t)1 << 12);
  seird_params params{};
  params.A = 0.0;
  seird_problem P = nullptr;
  seird_precond pc = nullptr;
  try {
    create_in_arena(m->mh, params, opts, part, *wo, a, &P, &pc);
  } catch (...) {
    throw;
  }
  // the objects' destructors must not free the fake addresses
  register_workspace(a.base, a.used + 1);
  if (pc) pc->prob = nullptr;
  delete pc;
  delete P;
  unregister_workspace(a.base);
  *bytes = (int64_t)a.used;
  API_END
}

seird_status seird_create_in_workspace(seird_mesh m, const seird_params *params, const seird_schwarz_opts *opts,
                                       const int32_t *part, const seird_workspace_opts *wo, void *ws,
                                       int64_t ws_bytes, seird_problem *prob, seird_precond *pc) {
  API_BEGIN
  if (!m || !params || !wo || !ws || !prob || (opts && (!part || !pc))) fail(SEIRD_ERR_ARG, "null argument");
  if (((uintptr_t)ws & 255) != 0) fail(SEIRD_ERR_ARG, "workspace must be 256-byte aligned");
  *prob = nullptr;
  if (pc) *pc = nullptr;
  Arena a;
  a.base = static_cast<uint8_t *>(ws);
  a.cap = (size_t)std::max<int64_t>(ws_bytes, 0);
  register_workspace(ws, a.cap);  // the creation's own reference, dropped below
  seird_problem P = nullptr;
  seird_precond C = nullptr;
  try {
    create_in_arena(m->mh, *params, opts, part, *wo, a, &P, &C);
  } catch (...) {
    unregister_workspace(ws);
    throw;
  }
  P->ws_base = ws;
  P->ws_bytes = a.cap;
  P->ws_restart = wo->restart_max;
  register_workspace(ws, a.cap);  // held by the problem
  if (C) {
    C->ws_base = ws;
    register_workspace(ws, a.cap);  // held by the preconditioner
  }
  unregister_workspace(ws);
  *prob = P;
  if (pc) *pc = C;
  API_END
}

void seird_problem_destroy(seird_problem p) { delete p; }

seird_status seird_set_params(seird_problem p, const seird_params *params) {
  API_BEGIN
  if (!p || !params) fail(SEIRD_ERR_ARG, "null argument");
  p->P = to_dev(*params);
  API_END
}

seird_status seird_set_beta_field(seird_problem p, const double *g_dev, void *stream) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  hipStream_t st = (hipStream_t)stream;
  if (!g_dev) {
    if (p->gfield != p->gfield_store) dev_free(p->gfield);
    p->gfield = nullptr;
  } else {
    if (!p->gfield) p->gfield = p->gfield_store ? p->gfield_store : dev_alloc<double>(p->mh.n);
    HIPCHECK(hipMemcpyAsync(p->gfield, g_dev, sizeof(double) * p->mh.n, hipMemcpyDeviceToDevice, st));
  }
  API_END
}

seird_status seird_set_beta_schedule(seird_problem p, const seird_beta_schedule *sch) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  if (p->md.inst) fail(SEIRD_ERR_ARG, "a batch's instances keep their own rates");
  p->sched = sch != nullptr;
  if (sch) {
    p->sa = sch->a;
    p->sb = sch->b;
    p->sk = sch->k;
    p->stc = sch->tc;
  }
  API_END
}

seird_status seird_set_time(seird_problem p, double t) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  p->time = t;
  API_END
}

seird_status seird_get_time(seird_problem p, double *t) {
  API_BEGIN
  if (!p || !t) fail(SEIRD_ERR_ARG, "null argument");
  *t = p->time;
  API_END
}

seird_status seird_set_mass(seird_problem p, int32_t consistent) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  if (consistent != 0 && consistent != 1) fail(SEIRD_ERR_ARG, "mass must be 0 (lumped) or 1 (consistent)");
  p->md.cmass_d = consistent ? p->d_cmass_d : nullptr;
  p->md.cmass_o = consistent ? p->d_cmass_o : nullptr;
  API_END
}

seird_status seird_set_boundary_flux(seird_problem p, const double *q_dev, void *stream) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  if (!q_dev) {
    p->md.qflux = nullptr;
  } else {
    HIPCHECK(hipMemcpyAsync(p->d_qflux, q_dev, sizeof(double) * 10 * p->mh.n, hipMemcpyDeviceToDevice,
                            (hipStream_t)stream));
    p->md.qflux = p->d_qflux;
  }
  API_END
}

seird_status seird_set_beta_regional(seird_problem p, double beta_c, double beta_e, double beta_w, double x_e,
                                     double x_w, double k_e, double k_w, void *stream) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  std::vector<double> g(p->mh.n);
  for (int64_t i = 0; i < p->mh.n; ++i) {
    const double x = p->mh.xy[2 * i];
    g[i] = beta_c + (beta_e - beta_c) / (1.0 + std::exp(-k_e * (x - x_e))) +
           (beta_w - beta_c) / (1.0 + std::exp(k_w * (x - x_w)));
  }
  if (!p->gfield) p->gfield = p->gfield_store ? p->gfield_store : dev_alloc<double>(p->mh.n);
  HIPCHECK(hipMemcpyAsync(p->gfield, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice, (hipStream_t)stream));
  HIPCHECK(hipStreamSynchronize((hipStream_t)stream));
  API_END
}

seird_status seird_problem_info(seird_problem p, int64_t *n_nodes, int64_t *n_slots) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  if (n_nodes) *n_nodes = p->mh.n;
  if (n_slots) *n_slots = (int64_t)p->mh.col.size();
  API_END
}

seird_status seird_pattern(seird_problem p, int64_t *rowptr, int32_t *col) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  if (rowptr) std::memcpy(rowptr, p->mh.rowptr.data(), sizeof(int64_t) * p->mh.rowptr.size());
  if (col) std::memcpy(col, p->mh.col.data(), sizeof(int32_t) * p->mh.col.size());
  API_END
}

seird_status seird_lumped_mass(seird_problem p, double *m_dev, void *stream) {
  API_BEGIN
  if (!p || !m_dev) fail(SEIRD_ERR_ARG, "null argument");
  HIPCHECK(hipMemcpyAsync(m_dev, p->md.mass, sizeof(double) * p->mh.n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  API_END
}

seird_status seird_residual(seird_problem p, const double *u, const double *u_prev, double dt, const double *src,
                            double *F, void *stream) {
  API_BEGIN
  if (!p || !u || !u_prev || !F) fail(SEIRD_ERR_ARG, "null argument");
  launch_residual(p->md, p->params_at(p->time), p->gfield, u, u_prev, dt, src, F, (hipStream_t)stream);
  HIPCHECK(hipGetLastError());
  API_END
}

seird_status seird_jacobian_size(seird_problem p, int64_t *n_vals) {
  API_BEGIN
  if (!p || !n_vals) fail(SEIRD_ERR_ARG, "null argument");
  *n_vals = p->nvals();
  API_END
}

seird_status seird_jacobian(seird_problem p, const double *u, double dt, double *vals, void *stream) {
  API_BEGIN
  if (!p || !u || !vals) fail(SEIRD_ERR_ARG, "null argument");
  launch_jacobian(p->md, p->params_at(p->time), p->gfield, u, dt, vals, vals + 25 * p->mh.n, (hipStream_t)stream);
  HIPCHECK(hipGetLastError());
  API_END
}

seird_status seird_spmv(seird_problem p, const double *vals, const double *x, double *y, int transpose,
                        void *stream) {
  API_BEGIN
  if (!p || !vals || !x || !y) fail(SEIRD_ERR_ARG, "null argument");
  launch_spmv(p->md, p->diag(vals), p->off(vals), x, nullptr, y, transpose, (hipStream_t)stream);
  HIPCHECK(hipGetLastError());
  API_END
}

static seird_precond precond_create_impl(seird_problem p, const seird_schwarz_opts *opts, const int32_t *part,
                                         int bs, const PrecondHost *proto);

seird_status seird_csr(seird_problem p, const int64_t **rowptr, const int32_t **col, int64_t *nnz,
                       int64_t *nrows) {
  API_BEGIN
  if (!p) fail(SEIRD_ERR_ARG, "null problem");
  if (!p->csr_ready) {
    if (p->ws_base && !p->csr_reserved)
      fail(SEIRD_ERR_WORKSPACE, "the workspace holds no CSR pattern (seird_workspace_opts.csr_pattern)");
    p->build_csr();
    p->csr_ready = true;
  }
  if (rowptr) *rowptr = p->csr_rowptr;
  if (col) *col = p->csr_col;
  if (nnz) *nnz = p->csr_nnz;
  if (nrows) *nrows = p->N;
  API_END
}

seird_status seird_csr_values(seird_problem p, const double *vals, double *csr_vals, void *stream) {
  API_BEGIN
  if (!p || !vals || !csr_vals) fail(SEIRD_ERR_ARG, "null argument");
  if (!p->csr_ready) fail(SEIRD_ERR_ARG, "call seird_csr first (it builds the pattern)");
  launch_csr_values(p->md, p->diag(vals), p->off(vals), p->csr_rowptr, csr_vals, (hipStream_t)stream);
  HIPCHECK(hipGetLastError());
  API_END
}

seird_status seird_precond_create(seird_problem p, const seird_schwarz_opts *opts, const int32_t *part,
                                  seird_precond *out) {
  API_BEGIN
  if (!p || !opts || !out) fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  *out = precond_create_impl(p, opts, part, NC);
  API_END
}

// Schwarz preconditioner of the coupled node-block Jacobian (bs = 5) or of
// one compartment's scalar matrix on the node graph (bs = 1, one-level).
static seird_precond precond_create_impl(seird_problem p, const seird_schwarz_opts *opts, const int32_t *part,
                                         int bs, const PrecondHost *proto) {
  auto pc = new seird_precond_s();
  try {
    pc->prob = p;
    pc->nvec = (int64_t)bs * p->mh.n;
    if (proto)  // the host structures of an identical preconditioner
      pc->ph = *proto;
    else
      build_precond(p->mh, *opts, part, pc->ph, bs);
    PrecondHost &ph = pc->ph;
    const int T = ph.tile;
    for (const SubInfo &s : ph.subs) {
      pc->max_nt = std::max(pc->max_nt, s.nt);
      pc->max_bu = std::max(pc->max_bu, s.bu);
    }
    if (T == 32 && pc->max_bu > 16)
      fail(SEIRD_ERR_ARG, "subdomain bandwidth above 16 tiles; use more subdomains");
    pc->sub_float = (T == 32 && ph.prec > 0);
    const size_t csz = pc->sub_float ? 4 : 8;
    // factorisation LDS: tile 32 three tiles (its U panel stays in
    // registers); tile 16 four staging tiles and the U panel
    const size_t lu_lds = T == 32 ? 3 * (size_t)T * (T + 1) * csz
                                  : 4 * (size_t)T * (T + 1) * csz + (size_t)pc->max_bu * T * (T + 1) * csz;
    if (lu_lds > p->lds_limit)
      fail(SEIRD_ERR_ARG, "subdomain bandwidth too large for the LDS of this device (" + std::to_string(lu_lds) +
                              " > " + std::to_string(p->lds_limit) + " bytes); use more subdomains or tile 16");
    for (const SubInfo &s : ph.subs)
      if (s.bl >= 32 || s.bu >= 32) fail(SEIRD_ERR_ARG, "subdomain block bandwidth must be below 32 tiles");
    if (ph.two_level && (ph.coarse.bl >= 32 || ph.coarse.bu >= 32))
      fail(SEIRD_ERR_ARG, "coarse block bandwidth must be below 32 tiles; use a coarser level or tile 32");
    if (pc->sub_float)
      pc->Fs = dev_alloc<float>(ph.factor_entries);
    else
      pc->Fs = dev_alloc<double>(ph.factor_entries);
    if (ph.prec == 1 && !pc->sub_float) pc->Fb = dev_alloc<float>(ph.factor_entries);
    if (ph.prec == 2) pc->Fb = dev_alloc<uint16_t>(ph.factor_entries);
    if (ph.two_level) pc->Fc = dev_alloc<double>(ph.coarse_entries);
    pc->subs_dev = dev_upload(ph.subs);
    pc->order_dev = dev_upload(ph.order);
    pc->ent_dev = dev_upload(ph.extract);
    pc->ent_ptr = dev_upload(ph.ent_ptr);
    pc->trow_ptr = dev_upload(ph.trow_ptr);
    pc->trow_sub = dev_upload(ph.trow_sub);
    pc->l2g = dev_upload(ph.l2g);
    pc->owned = dev_upload(ph.owned);
    pc->env_row = dev_upload(ph.env_row);
    pc->env_lo = dev_upload(ph.env_lo);
    pc->status = dev_alloc<int>(2);  // status flag, factorisation queue counter
    // transposed-apply gather lists: global unknown -> local copies
    {
      const int64_t N = pc->nvec;
      std::vector<int64_t> gptr(N + 1, 0);
      for (int32_t gidx : ph.l2g) gptr[gidx + 1]++;
      for (int64_t i = 0; i < N; ++i) gptr[i + 1] += gptr[i];
      std::vector<int32_t> gidx(ph.l2g.size());
      std::vector<int64_t> f(gptr.begin(), gptr.end() - 1);
      for (size_t l = 0; l < ph.l2g.size(); ++l) gidx[f[ph.l2g[l]]++] = (int32_t)l;
      pc->g2l_ptr = dev_upload(gptr);
      pc->g2l_idx = dev_upload(gidx);
      pc->yloc = dev_alloc<double>(ph.l2g.size());
    }
    pc->ybuf = dev_alloc<double>(ph.l2g.size());
    if (ph.two_level) {
      pc->coarse_dev = dev_upload(std::vector<SubInfo>{ph.coarse});
      pc->gp = dev_upload(ph.gal_p);
      pc->gq = dev_upload(ph.gal_q);
      pc->gptr = dev_upload(ph.gal_ptr);
      pc->gref = dev_upload(ph.gal_ref);
      pc->gw = dev_upload(ph.gal_w);
      pc->cperm = dev_upload(ph.c_perm);
      pc->z_ptr = dev_upload(ph.z_ptr);
      pc->z_col = dev_upload(ph.z_col);
      pc->z_val = dev_upload(ph.z_val);
      pc->zt_ptr = dev_upload(ph.zt_ptr);
      pc->zt_col = dev_upload(ph.zt_col);
      pc->zt_val = dev_upload(ph.zt_val);
      const int64_t cpad = (int64_t)ph.coarse.nt * T;
      pc->rc = dev_alloc<double>(cpad);
      pc->xc = dev_alloc<double>(cpad);
      pc->cscratch = dev_alloc<double>(cpad);
      if (!measuring()) HIPCHECK(hipMemset(pc->rc, 0, sizeof(double) * cpad));
      pc->t1 = dev_alloc<double>(p->N);
      if (T == 32 && coarse_inverse_bytes(ph.coarse.nt) <= COARSE_INVERSE_BUDGET) {
        const int64_t nt = ph.coarse.nt;
        // sized for the full inverses, so that any super-block size fits
        pc->Xc = dev_alloc<double>((size_t)(nt * (nt + 1) / 2) * 1024);
        pc->Wc = dev_alloc<double>((size_t)(nt * (nt + 1) / 2) * 1024);
        // the partial sums of a mat-vec over the largest block (any block size)
        pc->cpart = dev_alloc<double>((size_t)coarse_tri_chunks((int)nt) * T);
        pc->coarse_solver = 1;
        pc->coarse_block = (int)std::min<int64_t>(nt, std::max({COARSE_BLOCK, ph.coarse.bl, ph.coarse.bu}));
        pc->coarse_block_next = pc->coarse_block;
      }
      if (!measuring()) {
        HIPCHECK(hipStreamCreateWithFlags(&pc->st_coarse, hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&pc->ev_fork, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&pc->ev_join, hipEventDisableTiming));
        // first kernel and event on the stream now, so that the runtime's
        // own resources for them are set up at creation, not in a setup
        launch_fill_int(pc->status, 0, 2, pc->st_coarse);
        HIPCHECK(hipEventRecord(pc->ev_join, pc->st_coarse));
        HIPCHECK(hipEventSynchronize(pc->ev_join));
      }
    }
  } catch (...) {
    delete pc;
    throw;
  }
  return pc;
}

void seird_precond_destroy(seird_precond pc) { delete pc; }

seird_status seird_analyze_schwarz(int64_t n_nodes, const double *xy, int64_t n_tri, const int32_t *tri,
                                   const seird_schwarz_opts *opts, const int32_t *part, seird_schwarz_info *info,
                                   int32_t *l2g_out, uint8_t *owned_out) {
  API_BEGIN
  if (!opts || !info) fail(SEIRD_ERR_ARG, "null argument");
  MeshHost mh;
  build_mesh(n_nodes, xy, n_tri, tri, mh);
  PrecondHost ph;
  build_precond(mh, *opts, part, ph);
  info->factor_entries = ph.factor_entries + ph.coarse_entries;
  info->local_unknowns = (int64_t)ph.l2g.size();
  info->max_local_nodes = ph.max_nodes;
  info->max_bandwidth = ph.max_bw;
  info->mean_bandwidth = ph.mean_bw;
  info->coarse_n = ph.nc;
  info->coarse_bandwidth = ph.coarse_bw;
  info->lu_mfma_flops = ph.lu_mfma_flops;
  info->lu_useful_flops = ph.lu_useful_flops;
  if (l2g_out) std::memcpy(l2g_out, ph.l2g.data(), sizeof(int32_t) * ph.l2g.size());
  if (owned_out) std::memcpy(owned_out, ph.owned.data(), ph.owned.size());
  API_END
}

seird_status seird_precond_timing(seird_precond pc, int enable) {
  API_BEGIN
  if (!pc) fail(SEIRD_ERR_ARG, "null preconditioner");
  pc->timing = enable != 0;
  API_END
}

seird_status seird_precond_set_coarse_solver(seird_precond pc, int32_t solver) {
  API_BEGIN
  if (!pc) fail(SEIRD_ERR_ARG, "null preconditioner");
  if (solver < 0 || solver > 3) fail(SEIRD_ERR_ARG, "coarse solver must be 0, 1, 2 or 3");
  if (solver == 1 && !pc->Xc) fail(SEIRD_ERR_ARG, "no coarse inverses for this preconditioner");
  if (solver == 2 && !(pc->kc && pc->kc->cpc))
    fail(SEIRD_ERR_ARG, "no Krylov-RAS coarse solver (seird_precond_set_coarse_krylov)");
  if (solver == 3 && !(pc->kc && pc->kc->amg))
    fail(SEIRD_ERR_ARG, "no Krylov-AMG coarse solver (seird_precond_set_coarse_amg)");
  pc->coarse_solver = solver;
  pc->clear_graphs();
  API_END
}

seird_status seird_precond_set_coarse_block(seird_precond pc, int32_t tiles) {
  API_BEGIN
  if (!pc) fail(SEIRD_ERR_ARG, "null preconditioner");
  if (!pc->Xc) fail(SEIRD_ERR_ARG, "no coarse inverses for this preconditioner");
  const SubInfo &cs = pc->ph.coarse;
  if (tiles < 0) fail(SEIRD_ERR_ARG, "coarse block must be >= 0");
  const int S = tiles == 0 ? cs.nt : std::min(tiles, cs.nt);
  if (S < std::max(cs.bl, cs.bu))
    fail(SEIRD_ERR_ARG, "coarse block below the coarse band width (" + std::to_string(std::max(cs.bl, cs.bu)) +
                            " tile rows)");
  pc->coarse_block_next = S;  // the inverses in Xc/Wc keep their block until the next setup forms new ones
  API_END
}

seird_status seird_precond_set_solve_threads(seird_precond pc, int32_t threads) {
  API_BEGIN
  if (!pc) fail(SEIRD_ERR_ARG, "null preconditioner");
  const bool ok = threads == 256 || (pc->ph.tile == 32 && (threads == 128 || threads == 512 || threads == 1024));
  if (!ok) fail(SEIRD_ERR_ARG, "solve workgroup size must be 256, or 128/512/1024 with tile 32");
  pc->solve_threads = threads;
  pc->clear_graphs();
  API_END
}

seird_status seird_precond_info(seird_precond pc, int64_t *factor_entries, int64_t *coarse_n,
                                int32_t *max_local_nodes, int32_t *max_bandwidth) {
  API_BEGIN
  if (!pc) fail(SEIRD_ERR_ARG, "null preconditioner");
  if (factor_entries) *factor_entries = pc->ph.factor_entries + pc->ph.coarse_entries;
  if (coarse_n) *coarse_n = pc->ph.nc;
  if (max_local_nodes) *max_local_nodes = pc->ph.max_nodes;
  if (max_bandwidth) *max_bandwidth = pc->ph.max_bw;
  API_END
}

seird_status seird_precond_perf(seird_precond pc, seird_precond_perf_report *r, int reset) {
  API_BEGIN
  if (!pc || !r) fail(SEIRD_ERR_ARG, "null argument");
  const PrecondHost &ph = pc->ph;
  r->lu_mfma_flops = ph.lu_mfma_flops;
  r->lu_useful_flops = ph.lu_useful_flops;
  r->solve_bytes = pc->ras_bytes();
  r->factor_bytes = (double)ph.factor_entries * (pc->sub_float ? 4.0 : 8.0);
  r->setups = pc->set_count;
  r->t_extract_ms = pc->set_extract_ms;
  r->t_lu_ms = pc->set_lu_ms;
  if (reset) {
    pc->set_count = 0;
    pc->set_extract_ms = pc->set_lu_ms = 0.0;
  }
  API_END
}

static void precond_setup_raw(seird_precond pc, const double *diag, const double *off, hipStream_t st);
static int P_ncu(seird_precond pc) { return pc->prob->n_cu; }

static void precond_setup_impl(seird_precond pc, const double *vals, hipStream_t st) {
  seird_problem P = pc->prob;
  pc->vals_setup = vals;
  pc->kept_steps = -1;
  precond_setup_raw(pc, P->diag(vals), P->off(vals), st);
}

// setup from the matrix in node-block form (bs = 5: diag [n][25], off
// [slots][10]) or scalar form (bs = 1: diag [n], off [slots])
static void precond_setup_raw(seird_precond pc, const double *diag, const double *off, hipStream_t st) {
  PrecondHost &ph = pc->ph;
  HIPCHECK(hipMemsetAsync(pc->status, 0, sizeof(int), st));
  FactorLaunch fl;
  fl.tile = ph.tile;
  fl.bs = ph.bs;
  fl.Fs = pc->Fs;
  fl.sub_float = pc->sub_float;
  // bfloat16 factors: the float32 factorisation writes their copy itself
  fl.Fh = (ph.prec == 2 && pc->sub_float) ? pc->Fb : nullptr;
  fl.sub_entries = ph.factor_entries;
  fl.Fc = pc->Fc;
  fl.coarse_entries = ph.coarse_entries;
  fl.subs = pc->subs_dev;
  fl.erow = pc->env_row;
  fl.elo = pc->env_lo;
  fl.nsub = ph.n_sub;
  fl.order = pc->order_dev;
  fl.ent = pc->ent_dev;
  fl.ent_ptr = pc->ent_ptr;
  fl.trow_ptr = pc->trow_ptr;
  fl.trow_sub = pc->trow_sub;
  fl.ntrows = ph.trow_ptr.back();
  fl.max_node_blocks = ph.max_node_blocks;
  fl.max_bu = pc->max_bu;
  fl.status = pc->status;
  fl.queue = pc->status + 1;  // the int after the status flag
  fl.n_cu = P_ncu(pc);
  fl.dense_off = pc->dense_off;
  const bool krylov_coarse = ph.two_level && pc->coarse_solver >= 2;
  if (ph.two_level && !krylov_coarse) {
    fl.coarse = true;
    fl.cs = ph.coarse;
    fl.coarse_dev = pc->coarse_dev;
    fl.gp = pc->gp;
    fl.gq = pc->gq;
    fl.gptr = pc->gptr;
    fl.gref = pc->gref;
    fl.gw = pc->gw;
    fl.gal_nblk = (int64_t)ph.gal_p.size();
  }
  if (pc->timing) {
    for (hipEvent_t &e : pc->ev_set)
      if (!e) HIPCHECK(hipEventCreate(&e));
    fl.ev_extract = pc->ev_set[0];
    fl.ev_lu = pc->ev_set[1];
    fl.ev_lu_end = pc->ev_set[2];
  }
  if (ph.two_level && !krylov_coarse) {
    // fork: the coarse chain waits for everything already queued on st
    HIPCHECK(hipEventRecord(pc->ev_fork, st));
    HIPCHECK(hipStreamWaitEvent(pc->st_coarse, pc->ev_fork, 0));
    launch_setup_factors(fl, diag, off, st, pc->st_coarse);
    if (pc->Xc) {
      if (pc->coarse_block != pc->coarse_block_next) pc->clear_graphs();
      pc->coarse_block = pc->coarse_block_next;
      launch_coarse_inverse(pc->Fc, ph.coarse, pc->coarse_block, pc->Xc, pc->Wc, pc->st_coarse);
    }
    HIPCHECK(hipEventRecord(pc->ev_join, pc->st_coarse));
    HIPCHECK(hipStreamWaitEvent(st, pc->ev_join, 0));
  } else {
    launch_setup_factors(fl, diag, off, st, st);
  }
  HIPCHECK(hipGetLastError());
  pc->coarse_prepared = -1;
  if (krylov_coarse) {
    // Galerkin coarse matrix as node blocks of the coarse graph, then the
    // coarse RAS factors (no coarse factorisation)
    KrylovCoarse &kc = *pc->kc;
    const int64_t nc = ph.nc;
    launch_galerkin_blocks(kc.gdst, pc->gptr, pc->gref, pc->gw, (int64_t)ph.gal_p.size(), diag, off, kc.cvals,
                           kc.cvals + 25 * nc, st);
    if (kc.amg)
      amg_setup(*kc.amg, kc.cvals, kc.cvals + 25 * nc, pc->status, st);
    else
      precond_setup_raw(kc.cpc, kc.cvals, kc.cvals + 25 * nc, st);
  }
  if (pc->Fb && !fl.Fh) launch_convert(pc->Fb, ph.prec, pc->Fs, pc->sub_float ? 1 : 0, ph.factor_entries, st);
  int status = 0;
  HIPCHECK(hipMemcpyAsync(&status, pc->status, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (fl.ev_extract && ph.n_sub > 0) {
    float a = 0.f, b = 0.f;
    HIPCHECK(hipEventElapsedTime(&a, fl.ev_extract, fl.ev_lu));
    HIPCHECK(hipEventElapsedTime(&b, fl.ev_lu, fl.ev_lu_end));
    pc->set_extract_ms += a;
    pc->set_lu_ms += b;
    pc->set_count++;
  }
  pc->ready = true;
  if (ph.two_level) pc->coarse_prepared = krylov_coarse ? pc->coarse_solver : 0;
  if (status & 2) fail(SEIRD_ERR_ARG, "internal: local matrix entry outside the stored tiles");
  if (status) fail(SEIRD_ERR_BREAKDOWN, "zero or nonfinite pivot in a local LU factorisation");
}

seird_status seird_precond_setup_scalar(seird_precond pc, const double *diag, const double *off, void *stream) {
  API_BEGIN
  if (!pc || !diag || !off) fail(SEIRD_ERR_ARG, "null argument");
  if (pc->ph.bs != 1) fail(SEIRD_ERR_ARG, "not a scalar (compartment-wise) preconditioner");
  precond_setup_raw(pc, diag, off, (hipStream_t)stream);
  API_END
}

// greedy aggregation of a node graph (sorted neighbour lists, no self
// loops) in node order: (1) a node with no taken neighbour starts an
// aggregate with all its neighbours; (2) a free node joins the aggregate
// of its lowest-numbered neighbour taken in (1); (3) a node still free
// starts an aggregate with its free neighbours
static std::vector<int32_t> amg_aggregate(const std::vector<int64_t> &rp, const std::vector<int32_t> &cl,
                                          int64_t &na_out) {
  const int64_t n = (int64_t)rp.size() - 1;
  std::vector<int32_t> agg(n, -1);
  int32_t na = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free_nbrs = true;
    for (int64_t k = rp[i]; k < rp[i + 1] && free_nbrs; ++k) free_nbrs = agg[cl[k]] < 0;
    if (!free_nbrs) continue;
    agg[i] = na;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) agg[cl[k]] = na;
    ++na;
  }
  const std::vector<int32_t> first = agg;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
      if (first[cl[k]] >= 0) {
        agg[i] = first[cl[k]];
        break;
      }
  }
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
      if (agg[cl[k]] < 0) agg[cl[k]] = na;
    ++na;
  }
  na_out = na;
  return agg;
}

// The hierarchy's structure from the coarse graph (positions; perm maps
// original coarse numbers to positions).  The aggregation of level 0 runs
// in the original numbering (node order of the method), the later levels
// in aggregate order.
static AmgHier *amg_build(seird_problem C, const PrecondHost &ph, int max_coarse, int nu, double omega) {
  auto H = new AmgHier();
  try {
    H->nu = nu;
    H->omega = omega;
    const int64_t nc = ph.nc;
    std::vector<int32_t> pos_of = ph.c_perm, orig_of(nc);
    for (int64_t I = 0; I < nc; ++I) orig_of[pos_of[I]] = (int32_t)I;
    // level graph in the level's own node numbering (level 0: original)
    std::vector<int64_t> rp(nc + 1, 0);
    std::vector<int32_t> cl;
    for (int64_t I = 0; I < nc; ++I) {
      const int32_t p = pos_of[I];
      std::vector<int32_t> nb;
      for (int64_t k = ph.cg_rowptr[p]; k < ph.cg_rowptr[p + 1]; ++k) nb.push_back(orig_of[ph.cg_col[k]]);
      std::sort(nb.begin(), nb.end());
      cl.insert(cl.end(), nb.begin(), nb.end());
      rp[I + 1] = (int64_t)cl.size();
    }
    // device index of a level node: level 0 keeps positions, later levels the numbering itself
    std::vector<int32_t> dev_of(orig_of.size());
    for (int64_t I = 0; I < nc; ++I) dev_of[I] = pos_of[I];
    // level 0 device graph: the coarse problem's (positions)
    {
      AmgLevel L;
      L.n = nc;
      L.nslots = (int64_t)ph.cg_col.size();
      L.rowptr = C->md.rowptr;
      L.col = C->md.col;
      L.owns_graph = false;  // diag/off point into the Galerkin output, graph into the coarse problem
      H->lv.push_back(L);
    }
    // device slot of (device row, device column) for a level's device graph
    std::vector<int64_t> drp = ph.cg_rowptr;
    std::vector<int32_t> dcl = ph.cg_col;
    for (;;) {
      AmgLevel &L = H->lv.back();
      const int64_t n = L.n;
      if (n <= max_coarse) break;
      int64_t na = 0;
      const std::vector<int32_t> agg = amg_aggregate(rp, cl, na);
      if (na >= n) break;
      // next level graph (aggregates adjacent through any member edge), sorted
      std::vector<std::vector<int32_t>> nb(na);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
          if (agg[i] != agg[cl[k]]) nb[agg[i]].push_back(agg[cl[k]]);
      std::vector<int64_t> rp2(na + 1, 0);
      std::vector<int32_t> cl2;
      for (int64_t a = 0; a < na; ++a) {
        std::sort(nb[a].begin(), nb[a].end());
        nb[a].erase(std::unique(nb[a].begin(), nb[a].end()), nb[a].end());
        cl2.insert(cl2.end(), nb[a].begin(), nb[a].end());
        rp2[a + 1] = (int64_t)cl2.size();
      }
      // aggregate of each device node, members (ascending level numbering) per aggregate
      std::vector<int32_t> agg_dev(n);
      for (int64_t i = 0; i < n; ++i) agg_dev[dev_of[i]] = agg[i];
      std::vector<int64_t> aptr(na + 1, 0);
      for (int64_t i = 0; i < n; ++i) aptr[agg[i] + 1]++;
      for (int64_t a = 0; a < na; ++a) aptr[a + 1] += aptr[a];
      std::vector<int32_t> anodes(n);
      {
        std::vector<int64_t> f(aptr.begin(), aptr.end() - 1);
        for (int64_t i = 0; i < n; ++i) anodes[f[agg[i]]++] = dev_of[i];
      }
      // Galerkin map: every block of this level (device numbering) to its next-level block
      struct Src { int32_t dst; int32_t ref; };
      std::vector<Src> src;
      auto next_slot = [&](int32_t a, int32_t b) -> int32_t {
        const auto bg = cl2.begin() + rp2[a], en = cl2.begin() + rp2[a + 1];
        const auto it = std::lower_bound(bg, en, b);
        if (it == en || *it != b) fail(SEIRD_ERR_ARG, "internal: aggregate graph misses an edge");
        return (int32_t)(it - cl2.begin());
      };
      for (int64_t di = 0; di < n; ++di) {
        const int32_t a = agg_dev[di];
        src.push_back({-a - 1, (int32_t)(-di - 1)});
        for (int64_t k = drp[di]; k < drp[di + 1]; ++k) {
          const int32_t b = agg_dev[dcl[k]];
          src.push_back({a == b ? -a - 1 : next_slot(a, b), (int32_t)k});
        }
      }
      std::stable_sort(src.begin(), src.end(), [](const Src &x, const Src &y) { return x.dst < y.dst; });
      std::vector<int32_t> gdst, gref;
      std::vector<int64_t> gptr{0};
      for (size_t k = 0; k < src.size(); ++k) {
        if (k > 0 && src[k].dst != src[k - 1].dst) gptr.push_back((int64_t)gref.size());
        if (k == 0 || src[k].dst != src[k - 1].dst) gdst.push_back(src[k].dst);
        gref.push_back(src[k].ref);
      }
      gptr.push_back((int64_t)gref.size());
      L.nagg = na;
      L.agg = dev_upload(agg_dev);
      L.agg_ptr = dev_upload(aptr);
      L.agg_nodes = dev_upload(anodes);
      L.gdst = dev_upload(gdst);
      L.gptr = dev_upload(gptr);
      L.gref = dev_upload(gref);
      L.gnblk = (int64_t)gdst.size();
      AmgLevel N;
      N.n = na;
      N.nslots = (int64_t)cl2.size();
      N.rowptr = dev_upload(rp2);
      N.col = dev_upload(cl2);
      N.diag = dev_alloc<double>(25 * (size_t)na);
      N.off = dev_alloc<double>(25 * std::max<size_t>(cl2.size(), 1));
      H->lv.push_back(N);
      rp = rp2;
      cl = cl2;
      drp = rp2;
      dcl = cl2;
      dev_of.assign(na, 0);
      for (int64_t a = 0; a < na; ++a) dev_of[a] = (int32_t)a;
    }
    for (AmgLevel &L : H->lv) {
      L.dinv = dev_alloc<double>(25 * (size_t)L.n);
      L.x = dev_alloc<double>(5 * (size_t)L.n);
      L.b = dev_alloc<double>(5 * (size_t)L.n);
      L.r = dev_alloc<double>(5 * (size_t)L.n);
    }
    H->m_last = (int)(5 * H->lv.back().n);
    if (H->m_last > 4096) fail(SEIRD_ERR_ARG, "AMG last level too large for its dense inverse");
    H->Ainv = dev_alloc<double>((size_t)H->m_last * H->m_last);
  } catch (...) {
    delete H;
    throw;
  }
  return H;
}

// numeric setup: level 0's blocks are the Galerkin coarse matrix; the
// later levels are block sums; every level's diagonal blocks inverted; the
// last level's dense inverse by Gauss-Jordan with partial pivoting on the
// host
static void amg_setup(AmgHier &H, double *cdiag, double *coff, int *status, hipStream_t st) {
  H.lv[0].diag = cdiag;
  H.lv[0].off = coff;
  for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
    const AmgLevel &L = H.lv[l];
    AmgLevel &N = H.lv[l + 1];
    launch_galerkin_dense(L.gdst, L.gptr, L.gref, L.gnblk, L.diag, L.off, N.diag, N.off, st);
  }
  for (AmgLevel &L : H.lv) launch_block_inv5(L.n, L.diag, L.dinv, status, st);
  const AmgLevel &E = H.lv.back();
  std::vector<double> dg(25 * (size_t)E.n), of(25 * (size_t)E.nslots);
  std::vector<int64_t> rp(E.n + 1);
  std::vector<int32_t> cl(E.nslots);
  HIPCHECK(hipMemcpyAsync(dg.data(), E.diag, sizeof(double) * dg.size(), hipMemcpyDeviceToHost, st));
  if (E.nslots) HIPCHECK(hipMemcpyAsync(of.data(), E.off, sizeof(double) * of.size(), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(rp.data(), E.rowptr, sizeof(int64_t) * rp.size(), hipMemcpyDeviceToHost, st));
  if (E.nslots) HIPCHECK(hipMemcpyAsync(cl.data(), E.col, sizeof(int32_t) * cl.size(), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  const int m = H.m_last;
  std::vector<double> A((size_t)m * m, 0.0), X((size_t)m * m, 0.0);
  for (int64_t i = 0; i < E.n; ++i) {
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c < 5; ++c) A[(5 * i + r) * m + 5 * i + c] = dg[25 * i + 5 * r + c];
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
      for (int r = 0; r < 5; ++r)
        for (int c = 0; c < 5; ++c) A[(5 * i + r) * m + 5 * (int64_t)cl[k] + c] = of[25 * k + 5 * r + c];
  }
  for (int i = 0; i < m; ++i) X[(size_t)i * m + i] = 1.0;
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int r = k + 1; r < m; ++r)
      if (std::fabs(A[(size_t)r * m + k]) > std::fabs(A[(size_t)p * m + k])) p = r;
    const double piv = A[(size_t)p * m + k];
    if (!(std::fabs(piv) > 0.0) || !std::isfinite(piv))
      fail(SEIRD_ERR_BREAKDOWN, "singular last AMG level");
    if (p != k)
      for (int c = 0; c < m; ++c) {
        std::swap(A[(size_t)k * m + c], A[(size_t)p * m + c]);
        std::swap(X[(size_t)k * m + c], X[(size_t)p * m + c]);
      }
    const double rp_ = 1.0 / A[(size_t)k * m + k];
    for (int c = 0; c < m; ++c) {
      A[(size_t)k * m + c] *= rp_;
      X[(size_t)k * m + c] *= rp_;
    }
    for (int r = 0; r < m; ++r) {
      if (r == k) continue;
      const double f = A[(size_t)r * m + k];
      if (f == 0.0) continue;
      for (int c = 0; c < m; ++c) {
        A[(size_t)r * m + c] -= f * A[(size_t)k * m + c];
        X[(size_t)r * m + c] -= f * X[(size_t)k * m + c];
      }
    }
  }
  HIPCHECK(hipMemcpyAsync(H.Ainv, X.data(), sizeof(double) * X.size(), hipMemcpyHostToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));
}

// z = V(r) at level l (z, r of length 5 n_l): nu damped block-Jacobi sweeps
// from zero, coarse correction, nu sweeps; the last level's dense inverse
static void amg_vcycle(AmgHier &H, size_t l, const double *r, double *z, hipStream_t st) {
  AmgLevel &L = H.lv[l];
  if (l + 1 == H.lv.size()) {
    launch_dense_gemv(H.m_last, H.Ainv, r, z, st);
    return;
  }
  launch_fill(z, 0.0, 5 * L.n, st);
  for (int s = 0; s < H.nu; ++s) {
    launch_block_spmv(L.n, L.rowptr, L.col, L.diag, L.off, z, r, L.r, st);
    launch_block_jacobi(L.n, L.dinv, L.r, H.omega, z, st);
  }
  launch_block_spmv(L.n, L.rowptr, L.col, L.diag, L.off, z, r, L.r, st);
  AmgLevel &N = H.lv[l + 1];
  launch_agg_restrict(L.nagg, L.agg_ptr, L.agg_nodes, L.r, N.b, st);
  amg_vcycle(H, l + 1, N.b, N.x, st);
  launch_agg_prolong(L.n, L.agg, N.x, z, st);
  for (int s = 0; s < H.nu; ++s) {
    launch_block_spmv(L.n, L.rowptr, L.col, L.diag, L.off, z, r, L.r, st);
    launch_block_jacobi(L.n, L.dinv, L.r, H.omega, z, st);
  }
}

static void krylov_coarse_free(KrylovCoarse *kc) {
  if (!kc) return;
  delete kc->amg;
  delete kc->cpc;
  delete kc->cp;
  dev_free(kc->cvals);
  dev_free(kc->gdst);
  delete kc;
}

// inner GMRES on the coarse system, x0 = 0; an inner solve stopped by its
// iteration cap (or by its divergence test) returns its iterate
static void krylov_coarse_solve(seird_precond pc, const double *rc, double *xc, hipStream_t st) {
  KrylovCoarse &kc = *pc->kc;
  seird_problem C = kc.cp;
  const int64_t nc = C->mh.n;
  const double *cd = kc.cvals, *co = kc.cvals + 25 * nc;
  GmresOps ops;
  ops.N = 5 * nc;
  ops.seg = &C->seg;
  ops.seg_act = &C->seg_act;
  ops.seg_re = &C->seg_re;
  ops.spmv = [C, cd, co](const double *x, const double *b, double *y, hipStream_t s) {
    launch_block_spmv(C->md.n, C->md.rowptr, C->md.col, cd, co, x, b, y, s);
  };
  seird_precond cpc = kc.cpc;
  AmgHier *amg = kc.amg;
  if (amg)
    ops.prec = [amg](const double *r, double *z, hipStream_t s, const uint8_t *, const std::vector<uint8_t> *) {
      amg_vcycle(*amg, 0, r, z, s);
    };
  else
    ops.prec = [cpc](const double *r, double *z, hipStream_t s, const uint8_t *, const std::vector<uint8_t> *) {
      cpc->ras(r, z, 0, 0, s);
    };
  std::vector<seird_krylov_stats> stats;
  gmres_core(C, ops, rc, xc, kc.ko, stats, std::vector<uint8_t>{1}, st, KrylovWork{});
  kc.solves++;
  kc.its += stats[0].its;
  kc.its_max = std::max<int64_t>(kc.its_max, stats[0].its);
  if (stats[0].reason < 0) kc.unconverged++;
}

seird_status seird_precond_set_coarse_krylov(seird_precond pc, const seird_coarse_krylov_opts *o) {
  API_BEGIN
  if (!pc || !o) fail(SEIRD_ERR_ARG, "null argument");
  const PrecondHost &ph = pc->ph;
  if (!ph.two_level) fail(SEIRD_ERR_ARG, "the Krylov coarse solver needs a two-level preconditioner");
  if (o->restart < 1 || o->restart > KRYLOV_MAX - 1) fail(SEIRD_ERR_ARG, "inner restart must be in [1, 31]");
  if (o->max_it < 1) fail(SEIRD_ERR_ARG, "inner max_it must be >= 1");
  if (!(o->rtol >= 0.0) || !(o->atol >= 0.0)) fail(SEIRD_ERR_ARG, "inner tolerances must be >= 0");
  if (o->n_sub < 0 || o->overlap < 0) fail(SEIRD_ERR_ARG, "bad coarse subdomain options");
  const int64_t nc = ph.nc;
  // coarse subdomains: the fine subdomains' shares of the coarse nodes
  // (or n_sub groups of consecutive fine subdomain numbers), renumbered
  // over the non-empty ones
  const int nfine = ph.n_sub;
  std::vector<int32_t> grp(nc);
  for (int64_t p = 0; p < nc; ++p)
    grp[p] = o->n_sub > 0 ? (int32_t)((int64_t)ph.cg_owner[p] * o->n_sub / nfine) : ph.cg_owner[p];
  std::vector<int32_t> id(std::max(nfine, o->n_sub), -1);
  for (int64_t p = 0; p < nc; ++p) id[grp[p]] = 0;
  int nsc = 0;
  for (auto &v : id)
    if (v == 0) v = nsc++;
  for (int64_t p = 0; p < nc; ++p) grp[p] = id[grp[p]];
  MeshHost cm;
  cm.n = nc;
  cm.rowptr = ph.cg_rowptr;
  cm.col = ph.cg_col;
  cm.xy = ph.cg_xy;
  seird_schwarz_opts co{};
  co.n_sub = nsc;
  co.overlap = o->overlap;
  co.tile = ph.tile;
  co.factor_prec = 0;
  co.n_ref = 0;
  auto kc = new KrylovCoarse();
  try {
    kc->cp = problem_create_impl(cm, seird_params{});
    kc->cpc = precond_create_impl(kc->cp, &co, grp.data(), NC);
    kc->cpc->dense_off = true;
    kc->cvals = dev_alloc<double>((size_t)25 * (nc + (int64_t)ph.cg_col.size()));
    kc->gdst = dev_upload(ph.gal_dst);
    kc->cp->ensure_krylov(o->restart);
    kc->ko.restart = o->restart;
    kc->ko.max_it = o->max_it;
    kc->ko.rtol = o->rtol;
    kc->ko.atol = o->atol;
    kc->ko.dtol = 1e300;
    kc->ko.graphs = 0;
  } catch (...) {
    krylov_coarse_free(kc);
    throw;
  }
  krylov_coarse_free(pc->kc);
  pc->kc = kc;
  pc->coarse_solver = 2;
  pc->clear_graphs();
  API_END
}

seird_status seird_precond_set_coarse_amg(seird_precond pc, const seird_coarse_amg_opts *o) {
  API_BEGIN
  if (!pc || !o) fail(SEIRD_ERR_ARG, "null argument");
  const PrecondHost &ph = pc->ph;
  if (!ph.two_level) fail(SEIRD_ERR_ARG, "the Krylov coarse solver needs a two-level preconditioner");
  if (o->restart < 1 || o->restart > KRYLOV_MAX - 1) fail(SEIRD_ERR_ARG, "inner restart must be in [1, 31]");
  if (o->max_it < 1) fail(SEIRD_ERR_ARG, "inner max_it must be >= 1");
  if (!(o->rtol >= 0.0) || !(o->atol >= 0.0)) fail(SEIRD_ERR_ARG, "inner tolerances must be >= 0");
  if (o->max_coarse < 1 || o->max_coarse > 800) fail(SEIRD_ERR_ARG, "max_coarse must be in [1, 800]");
  if (o->nu < 1 || o->nu > 8) fail(SEIRD_ERR_ARG, "smoothing sweeps must be in [1, 8]");
  if (!(o->omega > 0.0 && o->omega < 2.0)) fail(SEIRD_ERR_ARG, "omega must be in (0, 2)");
  const int64_t nc = ph.nc;
  MeshHost cm;
  cm.n = nc;
  cm.rowptr = ph.cg_rowptr;
  cm.col = ph.cg_col;
  cm.xy = ph.cg_xy;
  auto kc = new KrylovCoarse();
  try {
    kc->cp = problem_create_impl(cm, seird_params{});
    kc->amg = amg_build(kc->cp, ph, o->max_coarse, o->nu, o->omega);
    kc->cvals = dev_alloc<double>((size_t)25 * (nc + (int64_t)ph.cg_col.size()));
    kc->gdst = dev_upload(ph.gal_dst);
    kc->cp->ensure_krylov(o->restart);
    kc->ko.restart = o->restart;
    kc->ko.max_it = o->max_it;
    kc->ko.rtol = o->rtol;
    kc->ko.atol = o->atol;
    kc->ko.dtol = 1e300;
    kc->ko.graphs = 0;
  } catch (...) {
    krylov_coarse_free(kc);
    throw;
  }
  krylov_coarse_free(pc->kc);
  pc->kc = kc;
  pc->coarse_solver = 3;
  pc->clear_graphs();
  API_END
}

seird_status seird_precond_coarse_krylov_stats(seird_precond pc, seird_coarse_krylov_stats *s, int reset) {
  API_BEGIN
  if (!pc || !s) fail(SEIRD_ERR_ARG, "null argument");
  if (!pc->kc) fail(SEIRD_ERR_ARG, "no Krylov coarse solver");
  KrylovCoarse &kc = *pc->kc;
  s->solves = kc.solves;
  s->its = kc.its;
  s->its_max = kc.its_max;
  s->unconverged = kc.unconverged;
  s->coarse_subdomains = kc.cpc ? kc.cpc->ph.n_sub : 0;
  s->coarse_local_unknowns = kc.cpc ? (int64_t)kc.cpc->ph.l2g.size() : 0;
  s->amg_levels = kc.amg ? (int32_t)kc.amg->lv.size() : 0;
  s->amg_last_nodes = kc.amg ? kc.amg->lv.back().n : 0;
  if (reset) kc.solves = kc.its = kc.its_max = kc.unconverged = 0;
  API_END
}

seird_status seird_precond_setup(seird_precond pc, const double *vals, void *stream) {
  API_BEGIN
  if (!pc || !vals) fail(SEIRD_ERR_ARG, "null argument");
  if (pc->ph.bs != NC) fail(SEIRD_ERR_ARG, "a scalar preconditioner is set up with seird_precond_setup_scalar");
  precond_setup_impl(pc, vals, (hipStream_t)stream);
  API_END
}

// ------------------------------------------------------------------------
// Autotuner cache: the chosen (tile, solve width) per (device architecture,
// kernel, shape bucket, factor precision), kept for the process and, when
// SEIRD_TUNE_CACHE names a file, in that file (one "key tile threads" line
// per entry, read on first use, appended on every new choice).
// ------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::string, std::pair<int, int>> g_tune_cache;
static bool g_tune_loaded = false;

static std::string tune_cache_file() {
  const char *e = std::getenv("SEIRD_TUNE_CACHE");
  return e ? std::string(e) : std::string();
}
static void tune_cache_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const std::string f = tune_cache_file();
  if (f.empty()) return;
  if (FILE *fp = std::fopen(f.c_str(), "r")) {
    char key[512];
    int tile = 0, th = 0;
    while (std::fscanf(fp, "%511s %d %d", key, &tile, &th) == 3) g_tune_cache[key] = {tile, th};
    std::fclose(fp);
  }
}
static bool tune_cache_get(const std::string &key, int &tile, int &th) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_cache_load_locked();
  auto it = g_tune_cache.find(key);
  if (it == g_tune_cache.end()) return false;
  tile = it->second.first;
  th = it->second.second;
  return true;
}
static void tune_cache_put(const std::string &key, int tile, int th) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_cache_load_locked();
  g_tune_cache[key] = {tile, th};
  const std::string f = tune_cache_file();
  if (f.empty()) return;
  if (FILE *fp = std::fopen(f.c_str(), "a")) {
    std::fprintf(fp, "%s %d %d\n", key.c_str(), tile, th);
    std::fclose(fp);
  }
}
// shape bucket: nodes per subdomain (log2), overlap, levels, precision
static std::string tune_key(const char *kernel, int device, int64_t n_nodes, int n_sub, int overlap, bool two_level,
                            int prec) {
  std::string arch = "unknown";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
  for (char &c : arch)
    if (c == ' ' || c == ':') c = '_';
  const int nb = (int)std::lround(std::log2(std::max<double>(1.0, (double)n_nodes / std::max(1, n_sub))));
  return arch + "|" + kernel + "|nodes_per_sub_2^" + std::to_string(nb) + "|overlap" + std::to_string(overlap) +
         (two_level ? "|two_level" : "|one_level") + "|prec" + std::to_string(prec);
}

seird_status seird_tune_cache_clear(void) {
  API_BEGIN
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache.clear();
  g_tune_loaded = true;  // a cleared cache does not reload its file
  API_END
}

seird_status seird_autotune_schwarz(seird_problem p, const seird_schwarz_opts *opts, const int32_t *part,
                                    const double *vals, int32_t applies_per_setup, int32_t reps,
                                    seird_tune_report *report, void *stream) {
  API_BEGIN
  if (!p || !opts || !part || !vals || !report) fail(SEIRD_ERR_ARG, "null argument");
  if (applies_per_setup < 1 || reps < 1) fail(SEIRD_ERR_ARG, "applies_per_setup and reps must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  using clk = std::chrono::steady_clock;
  *report = seird_tune_report{};
  const std::string key =
      tune_key("schwarz", p->device, p->mh.n, opts->n_sub, opts->overlap, opts->n_ref > 0, opts->factor_prec);
  {
    int tile = 0, th = 0;
    if (tune_cache_get(key, tile, th)) {
      report->best_tile = tile;
      report->best_solve_threads = th;
      report->from_cache = 1;
      return SEIRD_OK;
    }
  }
  std::vector<double> h(p->N);
  for (int64_t i = 0; i < p->N; ++i) h[i] = 1.0 + 0.5 * std::sin(0.37 * (double)i);
  struct Buffers {
    double *r = nullptr, *z = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Buffers() {
      dev_free(r);
      dev_free(z);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } B;
  B.r = dev_upload(h);
  B.z = dev_alloc<double>(p->N);
  HIPCHECK(hipEventCreate(&B.e0));
  HIPCHECK(hipEventCreate(&B.e1));
  double best = 0.0;
  int first_err = SEIRD_OK;
  std::string first_msg;
  auto add = [&](int tile, int th, int status, double set_ms, double app_ms) {
    if (report->n_candidates >= SEIRD_TUNE_MAX) return;
    seird_tune_candidate &c = report->cand[report->n_candidates++];
    c.tile = tile;
    c.solve_threads = th;
    c.status = status;
    c.setup_ms = set_ms;
    c.apply_ms = app_ms;
    c.score_ms = status == SEIRD_OK ? set_ms / applies_per_setup + app_ms : 0.0;
    if (status == SEIRD_OK && (report->best_tile == 0 || c.score_ms < best)) {
      best = c.score_ms;
      report->best_tile = tile;
      report->best_solve_threads = th;
    }
  };
  for (int tile : {32, 16}) {
    const std::vector<int> widths = tile == 32 ? std::vector<int>{256, 128, 512, 1024} : std::vector<int>{256};
    seird_schwarz_opts o = *opts;
    o.tile = tile;
    seird_precond pc = nullptr;
    const int rc = seird_precond_create(p, &o, part, &pc);
    if (rc != SEIRD_OK) {
      if (first_err == SEIRD_OK) {
        first_err = rc;
        first_msg = g_last_error;
      }
      for (int th : widths) add(tile, th, rc, 0.0, 0.0);
      continue;
    }
    std::unique_ptr<seird_precond_s> guard(pc);
    try {
      precond_setup_impl(pc, vals, st);  // warm-up (first launches load code)
      const auto t0 = clk::now();
      precond_setup_impl(pc, vals, st);  // synchronising
      const double set_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
      for (int th : widths) {
        pc->solve_threads = th;
        pc->apply(vals, B.r, B.z, 0, st);
        HIPCHECK(hipEventRecord(B.e0, st));
        for (int k = 0; k < reps; ++k) pc->apply(vals, B.r, B.z, 0, st);
        HIPCHECK(hipEventRecord(B.e1, st));
        HIPCHECK(hipEventSynchronize(B.e1));
        float t = 0.f;
        HIPCHECK(hipEventElapsedTime(&t, B.e0, B.e1));
        add(tile, th, SEIRD_OK, set_ms, (double)t / reps);
      }
    } catch (const Error &e) {
      if (e.code == SEIRD_ERR_HIP) throw;
      if (first_err == SEIRD_OK) {
        first_err = e.code;
        first_msg = e.msg;
      }
      for (int th : widths) add(tile, th, e.code, 0.0, 0.0);
    }
  }
  if (report->best_tile == 0) fail(SEIRD_ERR_ARG, "autotune: no candidate could be built (" + first_msg + ")");
  tune_cache_put(key, report->best_tile, report->best_solve_threads);
  API_END
}


seird_status seird_precond_apply(seird_precond pc, const double *r, double *z, int transpose, void *stream) {
  API_BEGIN
  if (!pc || !r || !z) fail(SEIRD_ERR_ARG, "null argument");
  // the two-grid apply multiplies by the Jacobian passed to the last setup,
  // which the caller keeps alive and unchanged
  pc->apply(pc->vals_setup, r, z, transpose, (hipStream_t)stream);
  HIPCHECK(hipGetLastError());
  API_END
}

seird_status seird_gmres(seird_problem p, seird_precond pc, const double *vals, const double *b, double *x,
                         const seird_krylov_opts *opts, seird_krylov_stats *stats, int transpose, void *stream) {
  API_BEGIN
  if (!p || !vals || !b || !x || !opts) fail(SEIRD_ERR_ARG, "null argument");
  std::vector<seird_krylov_stats> all;
  gmres_impl(p, pc, vals, b, x, *opts, all, std::vector<uint8_t>(p->seg.S, 1), transpose, (hipStream_t)stream);
  const int rc = all[0].reason < 0 ? all[0].reason : SEIRD_OK;
  if (stats) *stats = all[0];
  if (rc != SEIRD_OK) {
    g_last_error = rc == SEIRD_ERR_DIVERGED ? "GMRES diverged" : "GMRES reached max_it";
    return rc;
  }
  API_END
}

seird_status seird_gmres_noalloc(seird_problem p, seird_precond pc, const double *vals, const double *b, double *x,
                                 const seird_krylov_opts *opts, seird_krylov_stats *stats, int transpose,
                                 void *stream) {
  API_BEGIN
  if (!p || !vals || !b || !x || !opts) fail(SEIRD_ERR_ARG, "null argument");
  if (p->seg.S != 1) fail(SEIRD_ERR_ARG, "seird_gmres_noalloc takes a single problem");
  if (pc && pc->timing) fail(SEIRD_ERR_ARG, "seird_gmres_noalloc needs preconditioner timing off");
  const int m = opts->restart;
  if (m < 1 || m > KRYLOV_MAX - 1) fail(SEIRD_ERR_ARG, "restart must be in [1, 31]");
  // carve the static scratch: coefficient vector, reduction partials,
  // V [m+1][N], Z [m][N], each 256-byte aligned
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t hbytes = up(sizeof(double) * (size_t)p->HLD);
  const size_t pbytes = up(sizeof(double) * (size_t)p->seg.B * (KRYLOV_MAX + 2));
  const size_t vbytes = up(sizeof(double) * (size_t)(m + 1) * (size_t)p->N);
  const size_t zbytes = up(sizeof(double) * (size_t)m * (size_t)p->N);
  const size_t need = hbytes + pbytes + vbytes + zbytes;
  if (need > STATIC_SCRATCH_BYTES)
    fail(SEIRD_ERR_ARG, "seird_gmres_noalloc: restart " + std::to_string(m) + " with " + std::to_string(p->N) +
                            " unknowns needs " + std::to_string(need) + " bytes of scratch, above the " +
                            std::to_string((size_t)STATIC_SCRATCH_BYTES) +
                            " bytes of SEIRD_STATIC_SCRATCH_BYTES ((2 restart + 1) N 8 bytes plus a few KB)");
  unsigned char *base = (unsigned char *)static_scratch();
  KrylovWork w;
  w.hdev = (double *)base;
  w.partials = (double *)(base + hbytes);
  w.V = (double *)(base + hbytes + pbytes);
  w.Zb = (double *)(base + hbytes + pbytes + vbytes);
  seird_krylov_opts o = *opts;
  o.graphs = 0;  // graph instantiation allocates
  std::vector<seird_krylov_stats> all;
  gmres_impl(p, pc, vals, b, x, o, all, std::vector<uint8_t>(1, 1), transpose, (hipStream_t)stream, w);
  const int rc = all[0].reason < 0 ? all[0].reason : SEIRD_OK;
  if (stats) *stats = all[0];
  if (rc != SEIRD_OK) {
    g_last_error = rc == SEIRD_ERR_DIVERGED ? "GMRES diverged" : "GMRES reached max_it";
    return rc;
  }
  API_END
}

seird_status seird_step(seird_problem p, seird_precond pc, double *u, double dt, const double *src,
                        const seird_newton_opts *nopts, const seird_krylov_opts *kopts, seird_step_stats *stats,
                        void *stream) {
  seird_step_stats s{};
  int code = SEIRD_OK;
  try {
    std::vector<seird_step_stats> all;
    if (!p) fail(SEIRD_ERR_ARG, "null problem");
    step_impl(p, pc, u, dt, src, nopts, kopts, all, (hipStream_t)stream, p->time + dt);
    p->time += dt;
    if (!all.empty()) s = all[0];
  } catch (const Error &e) {
    code = e.code;
    g_last_error = e.msg;
  } catch (const std::exception &e) {
    code = SEIRD_ERR_ARG;
    g_last_error = std::string("internal: ") + e.what();
  }
  s.reason = code;
  if (stats) *stats = s;
  return code;
}

seird_status seird_forward_record(seird_problem p, seird_precond pc, double *u, int32_t n_steps, double dt,
                                  int32_t ckpt_every, const int32_t *region, int32_t n_regions, double *counts,
                                  const seird_newton_opts *nopts, const seird_krylov_opts *kopts, void *stream) {
  API_BEGIN
  if (!p || !u || !region || !counts || !nopts || !kopts) fail(SEIRD_ERR_ARG, "null argument");
  if (n_steps <= 0 || ckpt_every <= 0 || n_regions < 0) fail(SEIRD_ERR_ARG, "bad record sizes");
  hipStream_t st = (hipStream_t)stream;
  auto &T = p->tape;
  p->release_tape();
  ArenaScope tape_scope(p->tape_arena());  // a workspace problem records into its reserved pool
  const int64_t n = p->mh.n, N = p->N;
  // regions: per-node id and CSR of the nodes of each region
  std::vector<int64_t> rp(n_regions + 1, 0);
  for (int64_t j = 0; j < n; ++j) {
    if (region[j] >= n_regions) fail(SEIRD_ERR_ARG, "region id out of range");
    if (region[j] >= 0) rp[region[j] + 1]++;
  }
  for (int r = 0; r < n_regions; ++r) rp[r + 1] += rp[r];
  std::vector<int32_t> rn(rp[n_regions]);
  {
    std::vector<int64_t> f(rp.begin(), rp.end() - 1);
    for (int64_t j = 0; j < n; ++j)
      if (region[j] >= 0) rn[f[region[j]]++] = (int32_t)j;
  }
  T.region = dev_upload(std::vector<int32_t>(region, region + n));
  T.reg_ptr = dev_upload(rp);
  T.reg_nodes = dev_upload(rn);
  T.n_steps = n_steps;
  T.every = ckpt_every;
  T.n_regions = n_regions;
  T.dt = dt;
  T.t0 = p->time;
  // kept setups (pc_keep_steps) restart at every checkpoint: the first step
  // of a segment takes a fresh setup, here and when the reverse sweep
  // recomputes the segment, so that the recomputation repeats the recorded
  // steps exactly; the reverse sweep keeps its own transposed-solve setups
  // the same way
  T.nopts = *nopts;
  T.kopts = *kopts;
  const int n_seg = (n_steps + ckpt_every - 1) / ckpt_every;
  const int last0 = (n_seg - 1) * ckpt_every;  // first step index of the last segment
  for (int s = 0; s < n_seg; ++s) T.ckpt.push_back(dev_alloc<double>(N));
  for (int k = 0; k <= ckpt_every; ++k) T.seg.push_back(dev_alloc<double>(N));
  HIPCHECK(hipMemcpyAsync(T.ckpt[0], u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  if (last0 == 0) HIPCHECK(hipMemcpyAsync(T.seg[0], u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  for (int k = 1; k <= n_steps; ++k) {
    std::vector<seird_step_stats> s;
    if (pc && (k - 1) % ckpt_every == 0) pc->kept_steps = -1;  // a segment starts: fresh setup
    step_impl(p, pc, u, dt, nullptr, &T.nopts, kopts, s, st, T.t0 + k * dt);
    p->time = T.t0 + k * dt;
    launch_region_counts(T.reg_ptr, T.reg_nodes, p->md.mass, u, counts + (int64_t)(k - 1) * n_regions, n_regions, st);
    if (k % ckpt_every == 0 && k / ckpt_every < n_seg)
      HIPCHECK(hipMemcpyAsync(T.ckpt[k / ckpt_every], u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    if (k >= last0) HIPCHECK(hipMemcpyAsync(T.seg[k - last0], u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  }
  HIPCHECK(hipStreamSynchronize(st));
  T.seg_holds = n_seg - 1;
  T.valid = true;
  API_END
}

seird_status seird_adjoint(seird_problem p, seird_precond pc, const double *grad_counts, double *grad_g,
                           double *grad_nu, const seird_krylov_opts *kopts, seird_adjoint_stats *stats, void *stream) {
  API_BEGIN
  if (!p || !grad_counts || !grad_g || !grad_nu || !kopts) fail(SEIRD_ERR_ARG, "null argument");
  auto &T = p->tape;
  if (!T.valid) fail(SEIRD_ERR_ARG, "no forward record");
  hipStream_t st = (hipStream_t)stream;
  using clk = std::chrono::steady_clock;
  auto t_start = clk::now();
  seird_adjoint_stats as{};
  const int64_t n = p->mh.n, N = p->N;
  if (!T.lam) {
    ArenaScope tape_scope(p->tape_arena());
    T.lam = dev_alloc<double>(N);
    T.lam_next = dev_alloc<double>(N);
    T.rhs = dev_alloc<double>(N);
    T.partials = dev_alloc<double>(5 * ((n + 255) / 256) + 8);
  }
  HIPCHECK(hipMemsetAsync(T.lam_next, 0, sizeof(double) * N, st));
  HIPCHECK(hipMemsetAsync(grad_g, 0, sizeof(double) * n, st));
  double gnu[5] = {0, 0, 0, 0, 0};
  double *diag = p->vals, *off = p->vals + 25 * n;
  const int n_seg = (int)T.ckpt.size();
  std::vector<double> part;
  for (int s = n_seg - 1; s >= 0; --s) {
    const int n0 = s * T.every, n1 = std::min(T.n_steps, n0 + T.every);
    if (T.seg_holds != s) {  // recompute the states of this segment from its checkpoint
      T.seg_holds = -1;      // (a failure below leaves no segment marked as held)
      HIPCHECK(hipMemcpyAsync(T.seg[0], T.ckpt[s], sizeof(double) * N, hipMemcpyDeviceToDevice, st));
      for (int k = n0 + 1; k <= n1; ++k) {
        HIPCHECK(hipMemcpyAsync(T.seg[k - n0], T.seg[k - n0 - 1], sizeof(double) * N, hipMemcpyDeviceToDevice, st));
        std::vector<seird_step_stats> ss;
        if (pc && k == n0 + 1) pc->kept_steps = -1;  // as in the recorded run
        step_impl(p, pc, T.seg[k - n0], T.dt, nullptr, &T.nopts, &T.kopts, ss, st, T.t0 + k * T.dt);
        as.recomputed_steps++;
      }
      T.seg_holds = s;
    }
    // the transposed solves' setups: one per reverse step, or with
    // pc_keep_steps one serving that many further reverse steps of the
    // segment; a kept setup whose solve fails is rebuilt and the solve
    // repeated, and one that needs more than twice the iterations of its
    // fresh solve plus 5 is rebuilt at the next reverse step
    const int keep = pc ? T.nopts.pc_keep_steps : 0;
    int since = keep, fresh_its = 0;
    for (int k = n1; k > n0; --k) {
      const double *uk = T.seg[k - n0];
      const ParamsDev Pk = p->params_at(T.t0 + k * T.dt);
      launch_jacobian(p->md, Pk, p->gfield, uk, T.dt, diag, off, st);
      bool fresh = since >= keep;
      if (pc && fresh) {
        precond_setup_impl(pc, p->vals, st);
        as.setups++;
        since = 0;
      } else {
        ++since;
      }
      launch_adjoint_rhs(p->md, T.region, grad_counts + (int64_t)(k - 1) * T.n_regions, T.lam_next, T.rhs, st);
      for (;;) {
        std::vector<seird_krylov_stats> ks;
        gmres_impl(p, pc, p->vals, T.rhs, T.lam, *kopts, ks, std::vector<uint8_t>(p->seg.S, 1), 1, st);
        int its = 0, reason = 0;
        for (const auto &e : ks) {
          its += e.its;
          if (e.reason < 0) reason = e.reason;
        }
        as.gmres_its_total += its;
        if (reason < 0 && !fresh) {  // kept setup failed: rebuild and solve again
          precond_setup_impl(pc, p->vals, st);
          as.setups++;
          since = 0;
          fresh = true;
          continue;
        }
        if (reason < 0) fail(reason, "transposed GMRES failed in the adjoint sweep");
        if (fresh) fresh_its = its;
        else if (its > 2 * fresh_its + 5) since = keep;  // rebuild at the next reverse step
        break;
      }
      const int nb = launch_adjoint_grad(p->md, Pk, uk, T.lam, T.dt, grad_g, T.partials, st);
      part.resize(5 * (size_t)nb);
      HIPCHECK(hipMemcpyAsync(part.data(), T.partials, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      for (int c = 0; c < 5; ++c) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += part[(size_t)c * nb + b];
        gnu[c] -= T.dt * t;
      }
      std::swap(T.lam, T.lam_next);
    }
  }
  HIPCHECK(hipStreamSynchronize(st));
  for (int c = 0; c < 5; ++c) grad_nu[c] = gnu[c];
  as.t_reverse_ms = std::chrono::duration<double, std::milli>(clk::now() - t_start).count();
  if (stats) *stats = as;
  API_END
}

// ------------------------------------------------------------------------
// Decoupled Picard-Gauss-Seidel step (Appendix A, Eqs. weak_vec_implicit and
// picardtol): per sweep, the lagged scalar stiffness, then the compartments
// S, E, I, R, D one after the other, each a scalar system on the node graph
// solved in correction form by GMRES with a one-level RAS of scalar
// subdomains (a diagonal system, nu_c = 0, directly); stop when the sweep's
// update epsilon = ||u^{k+1} - u^k|| / ||u^n|| is at most tol.
// ------------------------------------------------------------------------
struct seird_pgs_s {
  seird_problem prob = nullptr;
  seird_precond pc = nullptr;  // bs = 1
  // kept per compartment (pc_lag), sharing pc's host structures; made on
  // first use from the creation's options and partition
  seird_precond lag[NC] = {};
  seird_schwarz_opts opts{};
  std::vector<int32_t> part;
  SegHost seg, seg_act, seg_re;  // one segment of n entries
  double *uk = nullptr, *Kd = nullptr, *Ko = nullptr, *sdiag = nullptr, *soff = nullptr, *r = nullptr,
         *delta = nullptr;
  ~seird_pgs_s() {
    for (seird_precond q : lag) delete q;
    delete pc;
    dev_free(seg.d_seg_start); dev_free(seg.d_blk_start); dev_free(seg.d_block_seg);
    dev_free(uk); dev_free(Kd); dev_free(Ko); dev_free(sdiag); dev_free(soff); dev_free(r); dev_free(delta);
  }
};

static void pgs_step_impl(seird_pgs g, double *u, double dt, const seird_pgs_opts &po, const seird_krylov_opts &ko,
                          seird_pgs_stats &stats, hipStream_t st) {
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  seird_problem p = g->prob;
  if (p->seg.S != 1) fail(SEIRD_ERR_ARG, "Picard-Gauss-Seidel steps take a single problem");
  if (po.max_sweeps < 1 || po.max_sweeps > SEIRD_MAX_PGS) fail(SEIRD_ERR_ARG, "max_sweeps out of range");
  const int64_t n = p->mh.n, N = p->N;
  const ParamsDev Pt = p->params_at(p->time + dt);  // coefficients at the end of the step
  stats = seird_pgs_stats{};
  HIPCHECK(hipMemcpyAsync(p->u_prev, u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  {
    HIPCHECK(hipMemsetAsync(p->flags, 0, sizeof(int), st));
    launch_check_state(u, n, nullptr, p->flags, st);
    int f = 0;
    HIPCHECK(hipMemcpyAsync(&f, p->flags, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (f & 1) fail(SEIRD_ERR_NONFINITE, "nonfinite state");
    if (f & 2) fail(SEIRD_ERR_STATE, "total density N <= 0 at a node");
  }
  const double unorm = p->seg_norms(p->u_prev, st)[0];
  GmresOps ops;
  ops.N = n;
  ops.seg = &g->seg;
  ops.seg_act = &g->seg_act;
  ops.seg_re = &g->seg_re;
  ops.spmv = [g](const double *x, const double *b, double *y, hipStream_t s) {
    launch_scalar_spmv(g->prob->md, g->sdiag, g->soff, x, b, y, s);
  };
  seird_precond cur = g->pc;  // the preconditioner of the compartment being solved
  ops.prec = [&cur](const double *r, double *z, hipStream_t s, const uint8_t *, const std::vector<uint8_t> *) {
    cur->apply(nullptr, r, z, 0, s);
  };
  seird_krylov_opts o = ko;
  o.graphs = 0;
  std::vector<seird_krylov_stats> ks;
  for (int k = 1;; ++k) {
    HIPCHECK(hipMemcpyAsync(g->uk, u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    launch_pgs_stiffness(p->md, g->uk, g->Kd, g->Ko, st);
    for (int c = 0; c < NC; ++c) {
      launch_pgs_system(p->md, Pt, p->gfield, c, dt, u, g->uk, p->u_prev, g->Kd, g->Ko, g->sdiag, g->soff, g->r,
                        st);
      if (Pt.nu[c] == 0.0 && !p->md.cmass_d) {  // lumped mass, no diffusion: a diagonal system
        launch_pgs_update(u, c, g->r, g->sdiag, n, st);
        continue;
      }
      auto t0 = clk::now();
      cur = g->pc;
      bool setup = true;
      if (po.pc_lag) {
        if (!g->lag[c]) g->lag[c] = precond_create_impl(p, &g->opts, g->part.data(), 1, &g->pc->ph);
        cur = g->lag[c];
        setup = k == 1;
      }
      if (setup) {
        precond_setup_raw(cur, g->sdiag, g->soff, st);
        stats.pc_setups++;
      }
      stats.t_setup_ms += std::chrono::duration<double, std::milli>(clk::now() - t0).count();
      t0 = clk::now();
      gmres_core(p, ops, g->r, g->delta, o, ks, std::vector<uint8_t>(1, 1), st, KrylovWork{});
      stats.t_gmres_ms += std::chrono::duration<double, std::milli>(clk::now() - t0).count();
      stats.gmres_its[c] += ks[0].its;
      if (ks[0].reason == SEIRD_ERR_DIVERGED) fail(SEIRD_ERR_DIVERGED, "GMRES diverged in compartment " + std::to_string(c));
      if (ks[0].reason == SEIRD_ERR_NOT_CONVERGED) {
        stats.inexact_solves++;
        if (po.strict_linear)
          fail(SEIRD_ERR_NOT_CONVERGED, "GMRES reached max_it in compartment " + std::to_string(c) + " of sweep " +
                                            std::to_string(k));
      }
      launch_pgs_update(u, c, g->delta, nullptr, n, st);
    }
    // epsilon of Eq. picardtol: ||u^{k+1} - u^k|| / ||u^n||
    HIPCHECK(hipMemcpyAsync(p->w1, g->uk, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    launch_axpby(p->w1, u, 1.0, nullptr, 0, -1.0, N, reduction_blocks(N), st);
    const double eps = p->seg_norms(p->w1, st)[0] / unorm;
    stats.eps_hist[k - 1] = eps;
    stats.sweeps = k;
    if (!std::isfinite(eps)) fail(SEIRD_ERR_NONFINITE, "nonfinite Picard-Gauss-Seidel update");
    if (eps <= po.tol) break;
    if (k >= po.max_sweeps)
      fail(SEIRD_ERR_NOT_CONVERGED, "Picard-Gauss-Seidel did not reach epsilon " + fmt_g(po.tol) + " in " +
                                        std::to_string(k) + " sweeps (last " + fmt_g(eps) + ")");
  }
  // the coupled residual of the result, scaled as the Newton stopping test
  launch_residual(p->md, Pt, p->gfield, u, p->u_prev, dt, nullptr, p->F, st);
  const double fn = p->seg_norms(p->F, st)[0];
  const double scale = p->seg_norms(p->u_prev, st, p->md.mass)[0];
  stats.res_scaled = fn / scale;
  stats.t_total_ms = std::chrono::duration<double, std::milli>(clk::now() - t_start).count();
}

struct seird_batch_s {
  seird_problem prob = nullptr;
  seird_precond pc = nullptr;
  std::vector<int64_t> node_off;
  ~seird_batch_s() {
    delete pc;
    delete prob;
  }
};

seird_status seird_pgs_create(seird_problem p, const seird_schwarz_opts *opts, const int32_t *part, seird_pgs *out) {
  API_BEGIN
  if (!p || !opts || !part || !out) fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  if (p->seg.S != 1) fail(SEIRD_ERR_ARG, "Picard-Gauss-Seidel steps take a single problem");
  if (opts->n_ref != 0) fail(SEIRD_ERR_ARG, "the compartment-wise preconditioner is one-level (n_ref = 0)");
  auto g = new seird_pgs_s();
  try {
    g->prob = p;
    g->pc = precond_create_impl(p, opts, part, 1);
    g->opts = *opts;
    g->part.assign(part, part + p->mh.n);
    const int64_t n = p->mh.n, ns = (int64_t)p->mh.col.size();
    SegHost sg;
    sg.S = 1;
    sg.seg_start = {0, n};
    sg.blk_start = {0, std::max<int64_t>(1, (n + SEG_CH - 1) / SEG_CH)};
    sg.B = (int)sg.blk_start[1];
    sg.block_seg.assign(sg.B, 0);
    sg.d_seg_start = dev_upload(sg.seg_start);
    sg.d_blk_start = dev_upload(sg.blk_start);
    sg.d_block_seg = dev_upload(sg.block_seg);
    g->seg = sg;
    g->seg_act = sg;
    g->seg_act.d_active = p->d_mask;
    g->seg_re = sg;
    g->seg_re.d_active = p->d_mask2;
    g->uk = dev_alloc<double>(p->N);
    g->Kd = dev_alloc<double>(n);
    g->Ko = dev_alloc<double>(ns);
    g->sdiag = dev_alloc<double>(n);
    g->soff = dev_alloc<double>(ns);
    g->r = dev_alloc<double>(n);
    g->delta = dev_alloc<double>(n);
  } catch (...) {
    delete g;
    throw;
  }
  *out = g;
  API_END
}

void seird_pgs_destroy(seird_pgs g) { delete g; }

seird_status seird_pgs_precond(seird_pgs g, seird_precond *out) {
  API_BEGIN
  if (!g || !out) fail(SEIRD_ERR_ARG, "null argument");
  *out = g->pc;
  API_END
}

seird_status seird_pgs_step(seird_pgs g, double *u, double dt, const seird_pgs_opts *popts,
                            const seird_krylov_opts *kopts, seird_pgs_stats *stats, void *stream) {
  seird_pgs_stats s{};
  int code = SEIRD_OK;
  try {
    if (!g || !u || !popts || !kopts) fail(SEIRD_ERR_ARG, "null argument");
    pgs_step_impl(g, u, dt, *popts, *kopts, s, (hipStream_t)stream);
    g->prob->time += dt;
  } catch (const Error &e) {
    code = e.code;
    g_last_error = e.msg;
  } catch (const std::exception &e) {
    code = SEIRD_ERR_ARG;
    g_last_error = std::string("internal: ") + e.what();
  }
  s.reason = code;
  if (stats) *stats = s;
  return code;
}

seird_status seird_batch_create(int32_t n_inst, const int64_t *n_nodes, const double *const *xy, const int64_t *n_tri,
                                const int32_t *const *tri, const seird_params *params, const int32_t *const *part,
                                const int32_t *n_sub, int32_t overlap, int32_t tile, int32_t factor_prec,
                                seird_batch *out) {
  API_BEGIN
  if (n_inst <= 0 || !n_nodes || !xy || !n_tri || !tri || !params || !part || !n_sub || !out)
    fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  auto B = new seird_batch_s();
  try {
    // concatenate the instances
    B->node_off.assign(n_inst + 1, 0);
    int64_t nt_total = 0;
    for (int k = 0; k < n_inst; ++k) {
      if (n_nodes[k] <= 0 || n_tri[k] <= 0) fail(SEIRD_ERR_ARG, "empty instance");
      B->node_off[k + 1] = B->node_off[k] + n_nodes[k];
      nt_total += n_tri[k];
    }
    const int64_t n = B->node_off[n_inst];
    std::vector<double> XY(2 * n);
    std::vector<int32_t> TRI(3 * nt_total), PART(n), INST(n);
    std::vector<ParamsDev> PI(n_inst);
    int64_t to = 0;
    int32_t so = 0;
    for (int k = 0; k < n_inst; ++k) {
      const int64_t o = B->node_off[k];
      std::copy(xy[k], xy[k] + 2 * n_nodes[k], XY.begin() + 2 * o);
      for (int64_t t = 0; t < 3 * n_tri[k]; ++t) {
        const int32_t v = tri[k][t];
        if (v < 0 || v >= n_nodes[k]) fail(SEIRD_ERR_MESH, "instance " + std::to_string(k) + ": vertex out of range");
        TRI[3 * to + t] = (int32_t)(v + o);
      }
      to += n_tri[k];
      for (int64_t j = 0; j < n_nodes[k]; ++j) {
        if (part[k][j] < 0 || part[k][j] >= n_sub[k]) fail(SEIRD_ERR_ARG, "partition entry out of range");
        PART[o + j] = part[k][j] + so;
        INST[o + j] = k;
      }
      so += n_sub[k];
      PI[k] = to_dev(params[k]);
    }
    seird_problem P = nullptr;
    int rc = seird_problem_create(n, XY.data(), nt_total, TRI.data(), &params[0], &P);
    if (rc != SEIRD_OK) fail(rc, g_last_error);
    B->prob = P;
    P->d_inst = dev_upload(INST);
    P->d_Pinst = dev_upload(PI);
    P->md.inst = P->d_inst;
    P->md.Pinst = P->d_Pinst;
    P->setup_segments(B->node_off);
    seird_schwarz_opts o{};
    o.n_sub = so;
    o.overlap = overlap;
    o.tile = tile;
    o.factor_prec = factor_prec;
    o.n_ref = 0;
    seird_precond pc = nullptr;
    rc = seird_precond_create(P, &o, PART.data(), &pc);
    if (rc != SEIRD_OK) fail(rc, g_last_error);
    B->pc = pc;
    std::vector<int32_t> sub_seg(so);
    for (int k = 0, s0 = 0; k < n_inst; s0 += n_sub[k], ++k)
      for (int j = 0; j < n_sub[k]; ++j) sub_seg[s0 + j] = k;
    pc->set_instances(sub_seg, n_inst);
  } catch (...) {
    delete B;
    throw;
  }
  *out = B;
  API_END
}

void seird_batch_destroy(seird_batch b) { delete b; }

seird_status seird_batch_info(seird_batch b, int64_t *node_offsets) {
  API_BEGIN
  if (!b || !node_offsets) fail(SEIRD_ERR_ARG, "null argument");
  std::copy(b->node_off.begin(), b->node_off.end(), node_offsets);
  API_END
}

seird_status seird_batch_precond(seird_batch b, seird_precond *out) {
  API_BEGIN
  if (!b || !out) fail(SEIRD_ERR_ARG, "null argument");
  *out = b->pc;
  API_END
}

seird_status seird_batch_step(seird_batch b, double *u, double dt, const seird_newton_opts *nopts,
                              const seird_krylov_opts *kopts, seird_step_stats *per_instance, void *stream) {
  API_BEGIN
  if (!b || !u) fail(SEIRD_ERR_ARG, "null argument");
  std::vector<seird_step_stats> all;
  step_impl(b->prob, b->pc, u, dt, nullptr, nopts, kopts, all, (hipStream_t)stream, b->prob->time + dt);
  b->prob->time += dt;
  if (per_instance) std::copy(all.begin(), all.end(), per_instance);
  API_END
}

seird_status seird_batch_autotune(seird_batch b, int32_t reps, seird_tune_report *report, void *stream) {
  API_BEGIN
  if (!b || !report) fail(SEIRD_ERR_ARG, "null argument");
  if (reps < 1) fail(SEIRD_ERR_ARG, "reps must be >= 1");
  seird_precond pc = b->pc;
  if (!pc->ready) fail(SEIRD_ERR_ARG, "batch autotune needs a set-up preconditioner (after a step)");
  hipStream_t st = (hipStream_t)stream;
  *report = seird_tune_report{};
  const int T = pc->ph.tile;
  const std::string key = tune_key("batch_schwarz_solve", b->prob->device, b->prob->mh.n, pc->ph.n_sub,
                                   pc->ph.overlap, false, pc->ph.prec) +
                          "|tile" + std::to_string(T);
  {
    int tile = 0, th = 0;
    if (tune_cache_get(key, tile, th)) {
      pc->solve_threads = th;
      pc->clear_graphs();
      report->best_tile = tile;
      report->best_solve_threads = th;
      report->from_cache = 1;
      return SEIRD_OK;
    }
  }
  const int64_t N = b->prob->N;
  std::vector<double> h(N);
  for (int64_t i = 0; i < N; ++i) h[i] = 1.0 + 0.5 * std::sin(0.37 * (double)i);
  double *r = dev_upload(h), *z = dev_alloc<double>(N);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 0.0;
  try {
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    const std::vector<int> widths = T == 32 ? std::vector<int>{256, 128, 512, 1024} : std::vector<int>{256};
    for (int th : widths) {
      pc->solve_threads = th;
      pc->ras(r, z, 0, 0, st);
      HIPCHECK(hipEventRecord(e0, st));
      for (int k = 0; k < reps; ++k) pc->ras(r, z, 0, 0, st);
      HIPCHECK(hipEventRecord(e1, st));
      HIPCHECK(hipEventSynchronize(e1));
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, e0, e1));
      seird_tune_candidate &c = report->cand[report->n_candidates++];
      c.tile = T;
      c.solve_threads = th;
      c.status = SEIRD_OK;
      c.apply_ms = c.score_ms = (double)t / reps;
      if (report->best_tile == 0 || c.score_ms < best) {
        best = c.score_ms;
        report->best_tile = T;
        report->best_solve_threads = th;
      }
    }
  } catch (...) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(r);
    dev_free(z);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dev_free(r);
  dev_free(z);
  pc->solve_threads = report->best_solve_threads;
  pc->clear_graphs();
  tune_cache_put(key, report->best_tile, report->best_solve_threads);
  API_END
}

}  // extern "C"

// ------------------------------------------------------------------------
// The 22-compartment model of Appendix C: decoupled Picard-Gauss-Seidel
// steps, one scalar system per compartment and sweep (Appendix A's
// iteration applied to Eqs. S ... D).
// ------------------------------------------------------------------------
namespace {
constexpr int NC22 = SEIRD22_NC;
// compartments whose loss rate d_c depends on the state (through lambda)
inline bool state_dependent_loss(int c) { return c == 0 || c == 1; }
inline double nu22(const seird22_params &p, int c) {
  static const int slot[NC22] = {0, 1, 2, -1, 3, -1, 4, 5, 6, -1, -1, -1, -1, -1, -1, -1, -1, -1, 8, 9, 7, -1};
  return slot[c] < 0 ? 0.0 : p.nu[slot[c]];
}
}  // namespace

struct seird22_s {
  seird_problem prob = nullptr;  // the mesh on the device, scalar Krylov basis and buffers
  seird22_params p{};
  seird_precond pc[NC22] = {};   // one-level scalar RAS of each diffusing compartment
  double pc_dt[NC22] = {};       // time step the preconditioner was set up for (0: never)
  SegHost seg, seg_act, seg_re;  // one segment of n entries (scalar systems)
  SegHost seg22;                 // one segment of 22 n entries (states)
  double *up = nullptr, *uk = nullptr, *w = nullptr, *Kd = nullptr, *Ko = nullptr, *sdiag = nullptr,
         *soff = nullptr, *r = nullptr, *delta = nullptr, *part22 = nullptr;
  int *flags = nullptr;
  ~seird22_s() {
    for (auto &q : pc) delete q;
    for (SegHost *g : {&seg, &seg22}) {
      dev_free(g->d_seg_start); dev_free(g->d_blk_start); dev_free(g->d_block_seg);
    }
    dev_free(up); dev_free(uk); dev_free(w); dev_free(Kd); dev_free(Ko); dev_free(sdiag); dev_free(soff);
    dev_free(r); dev_free(delta); dev_free(part22); dev_free(flags);
    delete prob;
  }
};

static SegHost one_segment(int64_t len) {
  SegHost sg;
  sg.S = 1;
  sg.seg_start = {0, len};
  sg.blk_start = {0, std::max<int64_t>(1, (len + SEG_CH - 1) / SEG_CH)};
  sg.B = (int)sg.blk_start[1];
  sg.block_seg.assign(sg.B, 0);
  sg.d_seg_start = dev_upload(sg.seg_start);
  sg.d_blk_start = dev_upload(sg.blk_start);
  sg.d_block_seg = dev_upload(sg.block_seg);
  return sg;
}

static void check22_params(const seird22_params &p) {
  const double *v = &p.beta_A;
  const size_t nv = sizeof(seird22_params) / sizeof(double);
  for (size_t k = 0; k < nv; ++k)
    if (!std::isfinite(v[k]) || v[k] < 0.0) fail(SEIRD_ERR_ARG, "22-compartment parameters must be finite and >= 0");
}

seird_status seird22_create(seird_mesh mesh, const seird22_params *p, const seird_schwarz_opts *opts,
                            const int32_t *part, seird22 *out) {
  API_BEGIN
  if (!mesh || !p || !opts || !part || !out) fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  if (opts->n_ref != 0) fail(SEIRD_ERR_ARG, "the compartment-wise preconditioner is one-level (n_ref = 0)");
  if (opts->factor_prec != 0) fail(SEIRD_ERR_ARG, "the compartment-wise preconditioner is FP64 (factor_prec = 0)");
  check22_params(*p);
  auto h = new seird22_s();
  try {
    h->p = *p;
    h->prob = problem_create_impl(mesh->mh, seird_params{});
    seird_problem P = h->prob;
    const int64_t n = P->mh.n, ns = (int64_t)P->mh.col.size();
    // every diffusing compartment gets its own preconditioner (also with
    // nu_c = 0, so that seird22_set_params may turn its diffusion on)
    int first = -1;
    for (int c = 0; c < NC22; ++c) {
      static const bool diffusing[NC22] = {1, 1, 1, 0, 1, 0, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 0};
      if (!diffusing[c]) continue;
      // the compartments share the subdomains: the host structures are built once
      h->pc[c] = precond_create_impl(P, opts, part, 1, first >= 0 ? &h->pc[first]->ph : nullptr);
      if (first < 0) first = c;
    }
    h->seg = one_segment(n);
    h->seg_act = h->seg;
    h->seg_act.d_active = P->d_mask;
    h->seg_re = h->seg;
    h->seg_re.d_active = P->d_mask2;
    h->seg22 = one_segment(NC22 * n);
    h->up = dev_alloc<double>(NC22 * n);
    h->uk = dev_alloc<double>(NC22 * n);
    h->w = dev_alloc<double>(NC22 * n);
    h->Kd = dev_alloc<double>(n);
    h->Ko = dev_alloc<double>(ns);
    h->sdiag = dev_alloc<double>(n);
    h->soff = dev_alloc<double>(ns);
    h->r = dev_alloc<double>(n);
    h->delta = dev_alloc<double>(n);
    h->part22 = dev_alloc<double>(h->seg22.B);
    h->flags = dev_alloc<int>(1);
    launch22_stiffness(P->md, h->Kd, h->Ko, nullptr);
    HIPCHECK(hipStreamSynchronize(nullptr));
  } catch (...) {
    delete h;
    throw;
  }
  *out = h;
  API_END
}

void seird22_destroy(seird22 h) { delete h; }

seird_status seird22_set_params(seird22 h, const seird22_params *p) {
  API_BEGIN
  if (!h || !p) fail(SEIRD_ERR_ARG, "null argument");
  check22_params(*p);
  h->p = *p;
  for (double &t : h->pc_dt) t = 0.0;  // the scalar matrices change: set up again
  API_END
}

seird_status seird22_residual(seird22 h, const double *u, const double *u_prev, double dt, double *F, void *stream) {
  API_BEGIN
  if (!h || !u || !u_prev || !F) fail(SEIRD_ERR_ARG, "null argument");
  launch22_residual(h->prob->md, h->p, u, u_prev, dt, F, (hipStream_t)stream);
  HIPCHECK(hipGetLastError());
  API_END
}

static void step22_impl(seird22 h, double *u, double dt, const seird_pgs_opts &po, const seird_krylov_opts &ko,
                        seird22_stats &stats, hipStream_t st) {
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  seird_problem P = h->prob;
  if (!(dt > 0.0)) fail(SEIRD_ERR_ARG, "dt must be > 0");
  if (po.max_sweeps < 1 || po.max_sweeps > SEIRD_MAX_PGS) fail(SEIRD_ERR_ARG, "max_sweeps out of range");
  const int64_t n = P->mh.n, N22 = NC22 * n;
  stats = seird22_stats{};
  HIPCHECK(hipMemcpyAsync(h->up, u, sizeof(double) * N22, hipMemcpyDeviceToDevice, st));
  {
    HIPCHECK(hipMemsetAsync(h->flags, 0, sizeof(int), st));
    launch22_check(u, N22, h->flags, st);
    int f = 0;
    HIPCHECK(hipMemcpyAsync(&f, h->flags, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (f) fail(SEIRD_ERR_NONFINITE, "nonfinite state");
  }
  auto norm22 = [&](const double *x) { return P->seg_norms(x, st, nullptr, h->part22, nullptr, &h->seg22)[0]; };
  const double unorm = norm22(h->up);
  GmresOps ops;
  ops.N = n;
  ops.seg = &h->seg;
  ops.seg_act = &h->seg_act;
  ops.seg_re = &h->seg_re;
  ops.spmv = [h](const double *x, const double *b, double *y, hipStream_t s) {
    launch_scalar_spmv(h->prob->md, h->sdiag, h->soff, x, b, y, s);
  };
  int cur = -1;  // compartment whose preconditioner the GMRES applies
  ops.prec = [h, &cur](const double *r, double *z, hipStream_t s, const uint8_t *, const std::vector<uint8_t> *) {
    h->pc[cur]->apply(nullptr, r, z, 0, s);
  };
  seird_krylov_opts o = ko;
  o.graphs = 0;
  std::vector<seird_krylov_stats> ks;
  for (int k = 1;; ++k) {
    HIPCHECK(hipMemcpyAsync(h->uk, u, sizeof(double) * N22, hipMemcpyDeviceToDevice, st));
    for (int c = 0; c < NC22; ++c) {
      launch22_system(P->md, h->p, c, dt, u, h->up, h->Kd, h->Ko, h->sdiag, h->r, st);
      const double coef = dt * nu22(h->p, c);
      if (coef == 0.0) continue;  // solved in place
      launch22_offdiag((int64_t)P->mh.col.size(), coef, h->Ko, h->soff, st);
      cur = c;
      const bool fresh = h->pc_dt[c] != dt || (state_dependent_loss(c) && k == 1);
      if (fresh) {
        auto t0 = clk::now();
        precond_setup_raw(h->pc[c], h->sdiag, h->soff, st);
        h->pc_dt[c] = dt;
        stats.pc_setups++;
        stats.t_setup_ms += std::chrono::duration<double, std::milli>(clk::now() - t0).count();
      }
      auto t0 = clk::now();
      gmres_core(P, ops, h->r, h->delta, o, ks, std::vector<uint8_t>(1, 1), st, KrylovWork{});
      stats.t_gmres_ms += std::chrono::duration<double, std::milli>(clk::now() - t0).count();
      stats.gmres_its[c] += ks[0].its;
      if (ks[0].reason == SEIRD_ERR_DIVERGED)
        fail(SEIRD_ERR_DIVERGED, "GMRES diverged in compartment " + std::to_string(c));
      if (ks[0].reason == SEIRD_ERR_NOT_CONVERGED) {
        stats.inexact_solves++;
        if (po.strict_linear)
          fail(SEIRD_ERR_NOT_CONVERGED, "GMRES reached max_it in compartment " + std::to_string(c));
      }
      launch22_update(u, c, h->delta, n, st);
    }
    // epsilon: ||u^{k+1} - u^k|| / ||u^n||
    HIPCHECK(hipMemcpyAsync(h->w, h->uk, sizeof(double) * N22, hipMemcpyDeviceToDevice, st));
    launch_axpby(h->w, u, 1.0, nullptr, 0, -1.0, N22, reduction_blocks(N22), st);
    const double eps = norm22(h->w) / unorm;
    stats.eps_hist[k - 1] = eps;
    stats.sweeps = k;
    if (!std::isfinite(eps)) fail(SEIRD_ERR_NONFINITE, "nonfinite Picard-Gauss-Seidel update");
    if (eps <= po.tol) break;
    if (k >= po.max_sweeps)
      fail(SEIRD_ERR_NOT_CONVERGED, "Picard-Gauss-Seidel did not reach epsilon " + fmt_g(po.tol) + " in " +
                                        std::to_string(k) + " sweeps (last " + fmt_g(eps) + ")");
  }
  launch22_residual(P->md, h->p, u, h->up, dt, h->w, st);
  const double fn = norm22(h->w);
  launch22_mass_scale(P->md.mass, h->up, h->w, n, st);
  stats.res_scaled = fn / norm22(h->w);
  stats.t_total_ms = std::chrono::duration<double, std::milli>(clk::now() - t_start).count();
}

seird_status seird22_step(seird22 h, double *u, double dt, const seird_pgs_opts *popts,
                          const seird_krylov_opts *kopts, seird22_stats *stats, void *stream) {
  seird22_stats s{};
  int code = SEIRD_OK;
  try {
    if (!h || !u || !popts || !kopts) fail(SEIRD_ERR_ARG, "null argument");
    step22_impl(h, u, dt, *popts, *kopts, s, (hipStream_t)stream);
  } catch (const Error &e) {
    code = e.code;
    g_last_error = e.msg;
  } catch (const std::exception &e) {
    code = SEIRD_ERR_ARG;
    g_last_error = std::string("internal: ") + e.what();
  }
  s.reason = code;
  if (stats) *stats = s;
  return code;
}
