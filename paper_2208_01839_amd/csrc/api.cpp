// C ABI of libseird and the host orchestration: Newton time step, restarted
// right-preconditioned GMRES, one-level and two-grid Schwarz apply.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "kernels.h"

using namespace seird;

namespace seird {
static thread_local std::string g_last_error;
[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }
void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(SEIRD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
void dev_free(void *p) {
  if (p) (void)hipFree(p);
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
  // adjoint record (checkpoints, last segment, regions)
  struct Tape {
    int n_steps = 0, every = 0, n_regions = 0;
    double dt = 0.0;
    seird_newton_opts nopts{};
    seird_krylov_opts kopts{};
    std::vector<double *> ckpt, seg;
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
      valid = false;
    }
  } tape;

  ~seird_problem_s() {
    dev_free(md.rowptr); dev_free(md.col); dev_free(md.tslot); dev_free(md.mass);
    dev_free(md.inc_ptr); dev_free(md.inc_j); dev_free(md.inc_l); dev_free(md.inc_sj); dev_free(md.inc_sl);
    dev_free(md.inc_K);
    dev_free(gfield); dev_free(partials); dev_free(hdev); dev_free(ydev); dev_free(flags);
    dev_free(u_prev); dev_free(F); dev_free(rhs); dev_free(delta); dev_free(vals);
    dev_free(V); dev_free(Zb); dev_free(w1);
    tape.release();
  }
  int64_t nvals() const { return 25 * mh.n + 10 * (int64_t)mh.col.size(); }
  const double *diag(const double *v) const { return v; }
  const double *off(const double *v) const { return v + 25 * mh.n; }

  double norm(const double *x, hipStream_t st, const double *scale = nullptr) {
    launch_norm2_partials(x, scale, N, partials, nb, st);
    launch_reduce(partials, nb, 1, hdev, st);
    double h;
    HIPCHECK(hipMemcpyAsync(&h, hdev, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    return std::sqrt(h);
  }
  void ensure_krylov(int m) {
    if (kcap >= m) return;
    dev_free(V); dev_free(Zb);
    V = dev_alloc<double>((size_t)(m + 1) * N);
    Zb = dev_alloc<double>((size_t)m * N);
    kcap = m;
  }
};

struct seird_precond_s {
  seird_problem prob = nullptr;
  PrecondHost ph;
  void *Fs = nullptr;        // subdomain factors as factorised (float64, or float32)
  bool sub_float = false;
  void *Fb = nullptr;        // bfloat16 copy for factor_prec 2, float32 copy for tile 16 + factor_prec 1
  double *Fc = nullptr;      // coarse factors (float64)
  SubInfo *subs_dev = nullptr;
  int32_t *order_dev = nullptr;
  ExtractEntry *ent_dev = nullptr;
  int32_t *l2g = nullptr;
  uint8_t *owned = nullptr;
  int *status = nullptr;
  int64_t *g2l_ptr = nullptr;
  int32_t *g2l_idx = nullptr;
  double *yloc = nullptr;
  int max_nt = 0, max_bu = 0;
  // coarse
  SubInfo *coarse_dev = nullptr;
  int32_t *gp = nullptr, *gq = nullptr, *gref = nullptr, *cperm = nullptr;
  int64_t *gptr = nullptr;
  double *gw = nullptr;
  int64_t *z_ptr = nullptr, *zt_ptr = nullptr;
  int32_t *z_col = nullptr, *zt_col = nullptr;
  double *z_val = nullptr, *zt_val = nullptr;
  double *rc = nullptr, *xc = nullptr, *cscratch = nullptr, *ybuf = nullptr;
  double *t1 = nullptr;
  const double *vals_setup = nullptr;  // Jacobian of the last setup (borrowed)
  bool ready = false;
  // second stream (default priority) for the coarse factorisation, which
  // runs concurrently with the subdomain factorisation
  hipStream_t st_coarse = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // optional HIP-event timing of the subdomain solve launches
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t ev_used = 0;
  double ras_ms = 0.0;
  int ras_count = 0;

  double ras_bytes() const {
    // algorithmic bytes of one subdomain-solve launch: every stored factor
    // entry once, plus per local unknown the index, the owner flag and the
    // gathered value, plus the owned results written
    const int64_t nsubent = ph.factor_entries;
    const double fsz = ph.prec == 0 ? 8.0 : (ph.prec == 1 ? 4.0 : 2.0);
    return nsubent * fsz + (double)ph.l2g.size() * (4 + 1 + 8) + (double)prob->N * 8;
  }
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
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (st_coarse) (void)hipStreamDestroy(st_coarse);
    for (auto &e : ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    dev_free(Fs); dev_free(Fb); dev_free(Fc); dev_free(subs_dev); dev_free(order_dev); dev_free(ent_dev); dev_free(l2g);
    dev_free(owned); dev_free(status); dev_free(g2l_ptr); dev_free(g2l_idx); dev_free(yloc);
    dev_free(coarse_dev); dev_free(gp); dev_free(gq); dev_free(gref); dev_free(cperm); dev_free(gptr); dev_free(gw);
    dev_free(z_ptr); dev_free(zt_ptr); dev_free(z_col); dev_free(zt_col); dev_free(z_val); dev_free(zt_val);
    dev_free(rc); dev_free(xc); dev_free(cscratch); dev_free(ybuf); dev_free(t1);
  }

  // factors read by the subdomain solves, in the storage precision ph.prec
  const void *factors() const {
    if (ph.prec == 0) return Fs;
    if (ph.prec == 1) return sub_float ? Fs : Fb;
    return Fb;
  }

  void ras(const double *r, double *z, int add, int transpose, hipStream_t st) {
    SolveLaunch sl;
    sl.tile = ph.tile;
    sl.prec = ph.prec;
    sl.F = factors();
    sl.subs = subs_dev;
    sl.order = order_dev;
    sl.nblocks = ph.n_sub;
    sl.l2g = l2g;
    sl.owned = owned;
    sl.r = r;
    sl.z = z;
    sl.add = add;
    sl.transpose = transpose;
    sl.yloc = yloc;
    sl.ybuf = ybuf;
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
    } else {
      launch_band_solve(sl, st);
    }
    if (transpose) launch_gather_copies(g2l_ptr, g2l_idx, yloc, z, add, prob->N, st);
  }

  // z += Z A_c^{-1} Z^T r  (or the transposed coarse operator)
  void coarse_add(const double *r, double *z, int transpose, hipStream_t st) {
    launch_coarse_restrict(zt_ptr, zt_col, zt_val, cperm, r, rc, ph.nc, st);
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

  void apply(const double *vals, const double *r, double *z, int transpose, hipStream_t st) {
    if (!ready) fail(SEIRD_ERR_ARG, "preconditioner used before setup");
    seird_problem P = prob;
    if (!ph.two_level) {
      ras(r, z, 0, transpose, st);
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
// GMRES (right preconditioned, restarted, CGS + one conditional DGKS pass)
// ------------------------------------------------------------------------
static int gmres_impl(seird_problem P, seird_precond pc, const double *vals, const double *b, double *x,
                      const seird_krylov_opts &o, seird_krylov_stats &stats, int transpose, hipStream_t st) {
  const int64_t N = P->N;
  const int m = o.restart;
  if (m < 1 || m > KRYLOV_MAX - 1) fail(SEIRD_ERR_ARG, "restart must be in [1, 31]");
  if (o.max_it < 0) fail(SEIRD_ERR_ARG, "max_it must be >= 0");
  P->ensure_krylov(m);
  const int nb = P->nb;
  double *V = P->V, *Zb = P->Zb;
  HIPCHECK(hipMemsetAsync(x, 0, sizeof(double) * N, st));
  const double bnorm = P->norm(b, st);
  stats = seird_krylov_stats{0, 0, bnorm, bnorm};
  if (!std::isfinite(bnorm)) fail(SEIRD_ERR_NONFINITE, "nonfinite right-hand side");
  const double target = std::max(o.rtol * bnorm, o.atol);
  if (bnorm <= target) {
    stats.reason = 1;
    return SEIRD_OK;
  }
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hbuf(KRYLOV_MAX + 4);
  double beta = bnorm;
  launch_axpby(V, b, 1.0 / beta, nullptr, 0, 0.0, N, nb, st);
  int its = 0;
  const double eta = 1.0 / std::sqrt(2.0);
  while (true) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    int reason = 0;
    for (int j = 0; j < m; ++j) {
      double *vj = V + (int64_t)j * N, *zj = Zb + (int64_t)j * N, *w = V + (int64_t)(j + 1) * N;
      if (pc)
        pc->apply(vals, vj, zj, transpose, st);
      else
        HIPCHECK(hipMemcpyAsync(zj, vj, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
      launch_spmv(P->md, P->diag(vals), P->off(vals), zj, nullptr, w, transpose, st);
      // h = V^T w, plus w.w
      launch_mdot(V, N, j + 1, w, N, 1, P->partials, nb, st);
      launch_reduce(P->partials, nb, j + 2, P->hdev, st);
      launch_maxpy_norm(w, V, N, P->hdev, j + 1, N, P->partials, nb, st);
      launch_reduce(P->partials, nb, 1, P->hdev + j + 2, st);
      HIPCHECK(hipMemcpyAsync(hbuf.data(), P->hdev, sizeof(double) * (j + 3), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      for (int i = 0; i <= j; ++i) H[i * m + j] = hbuf[i];
      const double wn0 = std::sqrt(hbuf[j + 1]);
      double wn = std::sqrt(hbuf[j + 2]);
      if (!std::isfinite(wn) || !std::isfinite(wn0)) fail(SEIRD_ERR_NONFINITE, "nonfinite Arnoldi vector");
      if (wn < eta * wn0) {  // DGKS: one reorthogonalisation pass
        launch_mdot(V, N, j + 1, w, N, 0, P->partials, nb, st);
        launch_reduce(P->partials, nb, j + 1, P->hdev, st);
        launch_maxpy_norm(w, V, N, P->hdev, j + 1, N, P->partials, nb, st);
        launch_reduce(P->partials, nb, 1, P->hdev + j + 1, st);
        HIPCHECK(hipMemcpyAsync(hbuf.data(), P->hdev, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        for (int i = 0; i <= j; ++i) H[i * m + j] += hbuf[i];
        wn = std::sqrt(hbuf[j + 1]);
      }
      H[(j + 1) * m + j] = wn;
      if (wn > 0.0) launch_axpby(w, w, 1.0 / wn, nullptr, 0, 0.0, N, nb, st);
      // Givens rotations
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t;
      }
      const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
      if (den == 0.0) {
        reason = 2;
        break;
      }
      cs[j] = H[j * m + j] / den;
      sn[j] = H[(j + 1) * m + j] / den;
      H[j * m + j] = den;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      k = j + 1;
      const double res = std::fabs(g[j + 1]);
      stats.resid = res;
      if (res < target) { reason = 1; break; }
      if (res > o.dtol * bnorm) { reason = SEIRD_ERR_DIVERGED; break; }
      if (its >= o.max_it) { reason = SEIRD_ERR_NOT_CONVERGED; break; }
      if (wn == 0.0) { reason = 2; break; }
    }
    if (k > 0) {
      for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int l = i + 1; l < k; ++l) s -= H[i * m + l] * y[l];
        y[i] = s / H[i * m + i];
      }
      HIPCHECK(hipMemcpyAsync(P->ydev, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
      launch_gemv_update(x, Zb, N, P->ydev, k, N, nb, st);
    }
    if (reason != 0) {
      stats.its = its;
      stats.reason = reason;
      HIPCHECK(hipStreamSynchronize(st));
      return reason > 0 ? SEIRD_OK : reason;
    }
    // restart from the true residual
    launch_spmv(P->md, P->diag(vals), P->off(vals), x, b, V, transpose, st);
    beta = P->norm(V, st);
    stats.resid = beta;
    if (beta <= target) {
      stats.its = its;
      stats.reason = 1;
      return SEIRD_OK;
    }
    launch_axpby(V, V, 1.0 / beta, nullptr, 0, 0.0, N, nb, st);
  }
}

static void precond_setup_impl(seird_precond pc, const double *vals, hipStream_t st);

static void step_impl(seird_problem p, seird_precond pc, double *u, double dt, const double *src,
                      const seird_newton_opts *nopts, const seird_krylov_opts *kopts, seird_step_stats &s,
                      hipStream_t st) {
  {
    if (!p || !u || !nopts || !kopts) fail(SEIRD_ERR_ARG, "null argument");
    if (nopts->max_it < 0 || nopts->max_it > SEIRD_MAX_NEWTON) fail(SEIRD_ERR_ARG, "Newton max_it out of range");
    if (nopts->pc_reuse < 0) fail(SEIRD_ERR_ARG, "pc_reuse must be >= 0");
    using clk = std::chrono::steady_clock;
    auto ms = [](clk::time_point a, clk::time_point b) {
      return std::chrono::duration<double, std::milli>(b - a).count();
    };
    const int64_t N = p->N;
    HIPCHECK(hipMemcpyAsync(p->u_prev, u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    auto check_state = [&](const double *x) {
      HIPCHECK(hipMemsetAsync(p->flags, 0, sizeof(int), st));
      launch_check_state(x, p->mh.n, p->flags, st);
      int f = 0;
      HIPCHECK(hipMemcpyAsync(&f, p->flags, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      if (f & 1) fail(SEIRD_ERR_NONFINITE, "nonfinite state");
      if (f & 2) fail(SEIRD_ERR_STATE, "total density N <= 0 at a node");
    };
    check_state(u);
    const double scale = p->norm(p->u_prev, st, p->md.mass);
    const double unorm = p->norm(p->u_prev, st);
    double *diag = p->vals, *off = p->vals + 25 * p->mh.n;
    int last_setup = 0, its_fresh = 0;
    bool stale = false;
    for (int k = 0;; ++k) {
      auto t0 = clk::now();
      launch_residual(p->md, p->P, p->gfield, u, p->u_prev, dt, src, p->F, st);
      const double fn = p->norm(p->F, st);
      s.t_residual_ms += ms(t0, clk::now());
      s.res_hist[k] = fn / scale;
      if (!std::isfinite(fn)) fail(SEIRD_ERR_NONFINITE, "nonfinite residual");
      if (fn <= nopts->tol * scale) break;
      if (k >= nopts->max_it) fail(SEIRD_ERR_NOT_CONVERGED, "Newton did not converge");
      t0 = clk::now();
      launch_jacobian(p->md, p->P, p->gfield, u, dt, diag, off, st);
      HIPCHECK(hipStreamSynchronize(st));
      s.t_jacobian_ms += ms(t0, clk::now());
      // preconditioner setup: fresh at the first iteration, then every
      // pc_reuse + 1 iterations, or when the reused one was marked stale
      t0 = clk::now();
      bool fresh = false;
      if (pc && (k == 0 || stale || (k - last_setup) > nopts->pc_reuse)) {
        precond_setup_impl(pc, p->vals, st);
        s.pc_setups++;
        last_setup = k;
        stale = false;
        fresh = true;
      }
      s.t_setup_ms += ms(t0, clk::now());
      t0 = clk::now();
      launch_axpby(p->rhs, p->F, -1.0, nullptr, 0, 0.0, N, p->nb, st);
      seird_krylov_stats ks{};
      int rc = gmres_impl(p, pc, p->vals, p->rhs, p->delta, *kopts, ks, 0, st);
      if (pc && !fresh && rc != SEIRD_OK) {
        // a reused setup failed: rebuild it from the current Jacobian and retry
        auto t1 = clk::now();
        precond_setup_impl(pc, p->vals, st);
        s.pc_setups++;
        last_setup = k;
        s.t_setup_ms += ms(t1, clk::now());
        const int its_first = ks.its;
        rc = gmres_impl(p, pc, p->vals, p->rhs, p->delta, *kopts, ks, 0, st);
        ks.its += its_first;
        fresh = true;
      }
      if (fresh) its_fresh = ks.its;
      else if (ks.its > 2 * its_fresh + 5) stale = true;  // reuse no longer pays
      s.t_gmres_ms += ms(t0, clk::now());
      if (pc && pc->timing) {
        HIPCHECK(hipStreamSynchronize(st));
        pc->harvest();
      }
      s.gmres_its[k] = ks.its;
      s.gmres_its_total += ks.its;
      s.newton_its = k + 1;
      if (rc == SEIRD_ERR_DIVERGED) fail(rc, "GMRES diverged");
      // max_it without convergence: inexact Newton update is still taken
      launch_axpby(u, p->delta, 1.0, nullptr, 0, 1.0, N, p->nb, st);
      s.eps = p->norm(p->delta, st) / unorm;
      check_state(u);
    }
    if (pc && pc->timing) {
      s.t_ras_kernel_ms = pc->ras_ms;
      s.n_ras_launches = pc->ras_count;
      s.ras_bytes_per_launch = pc->ras_bytes();
      pc->ras_ms = 0.0;
      pc->ras_count = 0;
    }
  }
}


extern "C" {

const char *seird_last_error(void) { return g_last_error.c_str(); }
const char *seird_version(void) { return "libseird 0.1 gfx950"; }

seird_status seird_problem_create(int64_t n_nodes, const double *xy, int64_t n_tri, const int32_t *tri,
                                  const seird_params *params, seird_problem *out) {
  API_BEGIN
  if (!out || !params) fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  auto P = new seird_problem_s();
  try {
    HIPCHECK(hipGetDevice(&P->device));
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) == hipSuccess && lds > 0)
      P->lds_limit = (size_t)lds;
    build_mesh(n_nodes, xy, n_tri, tri, P->mh);
    P->P = to_dev(*params);
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
    P->md.inc_sl = dev_upload(m.inc_sl);
    P->md.inc_K = dev_upload(m.inc_K);
    P->N = 5 * m.n;
    P->nb = reduction_blocks(P->N);
    P->partials = dev_alloc<double>((size_t)P->nb * (KRYLOV_MAX + 2));
    P->hdev = dev_alloc<double>(KRYLOV_MAX + 8);
    P->ydev = dev_alloc<double>(KRYLOV_MAX + 8);
    P->flags = dev_alloc<int>(4);
    P->u_prev = dev_alloc<double>(P->N);
    P->F = dev_alloc<double>(P->N);
    P->rhs = dev_alloc<double>(P->N);
    P->delta = dev_alloc<double>(P->N);
    P->w1 = dev_alloc<double>(P->N);
    P->vals = dev_alloc<double>(P->nvals());
  } catch (...) {
    delete P;
    throw;
  }
  *out = P;
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
    dev_free(p->gfield);
    p->gfield = nullptr;
  } else {
    if (!p->gfield) p->gfield = dev_alloc<double>(p->mh.n);
    HIPCHECK(hipMemcpyAsync(p->gfield, g_dev, sizeof(double) * p->mh.n, hipMemcpyDeviceToDevice, st));
  }
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
  launch_residual(p->md, p->P, p->gfield, u, u_prev, dt, src, F, (hipStream_t)stream);
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
  launch_jacobian(p->md, p->P, p->gfield, u, dt, vals, vals + 25 * p->mh.n, (hipStream_t)stream);
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

seird_status seird_precond_create(seird_problem p, const seird_schwarz_opts *opts, const int32_t *part,
                                  seird_precond *out) {
  API_BEGIN
  if (!p || !opts || !out) fail(SEIRD_ERR_ARG, "null argument");
  *out = nullptr;
  auto pc = new seird_precond_s();
  try {
    pc->prob = p;
    build_precond(p->mh, *opts, part, pc->ph);
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
    const size_t lu_lds = 4 * (size_t)T * (T + 1) * csz + (size_t)pc->max_bu * T * (T + 1) * csz;
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
    pc->l2g = dev_upload(ph.l2g);
    pc->owned = dev_upload(ph.owned);
    pc->status = dev_alloc<int>(1);
    // transposed-apply gather lists: global unknown -> local copies
    {
      const int64_t N = p->N;
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
      HIPCHECK(hipMemset(pc->rc, 0, sizeof(double) * cpad));
      pc->t1 = dev_alloc<double>(p->N);
      HIPCHECK(hipStreamCreateWithFlags(&pc->st_coarse, hipStreamNonBlocking));
      HIPCHECK(hipEventCreateWithFlags(&pc->ev_fork, hipEventDisableTiming));
      HIPCHECK(hipEventCreateWithFlags(&pc->ev_join, hipEventDisableTiming));
    }
  } catch (...) {
    delete pc;
    throw;
  }
  *out = pc;
  API_END
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

static void precond_setup_impl(seird_precond pc, const double *vals, hipStream_t st) {
  seird_problem P = pc->prob;
  PrecondHost &ph = pc->ph;
  HIPCHECK(hipMemsetAsync(pc->status, 0, sizeof(int), st));
  FactorLaunch fl;
  fl.tile = ph.tile;
  fl.Fs = pc->Fs;
  fl.sub_float = pc->sub_float;
  fl.sub_entries = ph.factor_entries;
  fl.Fc = pc->Fc;
  fl.coarse_entries = ph.coarse_entries;
  fl.subs = pc->subs_dev;
  fl.nsub = ph.n_sub;
  fl.order = pc->order_dev;
  fl.ent = pc->ent_dev;
  fl.nent = (int64_t)ph.extract.size();
  fl.max_bu = pc->max_bu;
  fl.status = pc->status;
  if (ph.two_level) {
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
  if (ph.two_level) {
    // fork: the coarse chain waits for everything already queued on st
    HIPCHECK(hipEventRecord(pc->ev_fork, st));
    HIPCHECK(hipStreamWaitEvent(pc->st_coarse, pc->ev_fork, 0));
    launch_setup_factors(fl, P->diag(vals), P->off(vals), st, pc->st_coarse);
    HIPCHECK(hipEventRecord(pc->ev_join, pc->st_coarse));
    HIPCHECK(hipStreamWaitEvent(st, pc->ev_join, 0));
  } else {
    launch_setup_factors(fl, P->diag(vals), P->off(vals), st, st);
  }
  HIPCHECK(hipGetLastError());
  if (pc->Fb) launch_convert(pc->Fb, ph.prec, pc->Fs, pc->sub_float ? 1 : 0, ph.factor_entries, st);
  int status = 0;
  HIPCHECK(hipMemcpyAsync(&status, pc->status, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  pc->ready = true;
  pc->vals_setup = vals;
  if (status & 2) fail(SEIRD_ERR_ARG, "internal: local matrix entry outside the tile band");
  if (status) fail(SEIRD_ERR_BREAKDOWN, "zero or nonfinite pivot in a local LU factorisation");
}

seird_status seird_precond_setup(seird_precond pc, const double *vals, void *stream) {
  API_BEGIN
  if (!pc || !vals) fail(SEIRD_ERR_ARG, "null argument");
  precond_setup_impl(pc, vals, (hipStream_t)stream);
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
  seird_krylov_stats s{};
  int rc = gmres_impl(p, pc, vals, b, x, *opts, s, transpose, (hipStream_t)stream);
  if (stats) *stats = s;
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
    step_impl(p, pc, u, dt, src, nopts, kopts, s, (hipStream_t)stream);
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
  T.release();
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
  T.nopts = *nopts;
  T.kopts = *kopts;
  const int n_seg = (n_steps + ckpt_every - 1) / ckpt_every;
  const int last0 = (n_seg - 1) * ckpt_every;  // first step index of the last segment
  for (int s = 0; s < n_seg; ++s) T.ckpt.push_back(dev_alloc<double>(N));
  for (int k = 0; k <= ckpt_every; ++k) T.seg.push_back(dev_alloc<double>(N));
  HIPCHECK(hipMemcpyAsync(T.ckpt[0], u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  if (last0 == 0) HIPCHECK(hipMemcpyAsync(T.seg[0], u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  for (int k = 1; k <= n_steps; ++k) {
    seird_step_stats s{};
    step_impl(p, pc, u, dt, nullptr, nopts, kopts, s, st);
    launch_region_counts(T.reg_ptr, T.reg_nodes, p->md.mass, u, counts + (int64_t)(k - 1) * n_regions, n_regions, st);
    if (k % ckpt_every == 0 && k / ckpt_every < n_seg)
      HIPCHECK(hipMemcpyAsync(T.ckpt[k / ckpt_every], u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    if (k >= last0) HIPCHECK(hipMemcpyAsync(T.seg[k - last0], u, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  }
  HIPCHECK(hipStreamSynchronize(st));
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
    if (s < n_seg - 1) {  // recompute the states of this segment from its checkpoint
      HIPCHECK(hipMemcpyAsync(T.seg[0], T.ckpt[s], sizeof(double) * N, hipMemcpyDeviceToDevice, st));
      for (int k = n0 + 1; k <= n1; ++k) {
        HIPCHECK(hipMemcpyAsync(T.seg[k - n0], T.seg[k - n0 - 1], sizeof(double) * N, hipMemcpyDeviceToDevice, st));
        seird_step_stats ss{};
        step_impl(p, pc, T.seg[k - n0], T.dt, nullptr, &T.nopts, &T.kopts, ss, st);
        as.recomputed_steps++;
      }
    }
    for (int k = n1; k > n0; --k) {
      const double *uk = T.seg[k - n0];
      launch_jacobian(p->md, p->P, p->gfield, uk, T.dt, diag, off, st);
      if (pc) precond_setup_impl(pc, p->vals, st);
      launch_adjoint_rhs(p->md.mass, T.region, grad_counts + (int64_t)(k - 1) * T.n_regions, T.lam_next, T.rhs, n, st);
      seird_krylov_stats ks{};
      int rc = gmres_impl(p, pc, p->vals, T.rhs, T.lam, *kopts, ks, 1, st);
      as.gmres_its_total += ks.its;
      if (rc != SEIRD_OK) fail(rc, "transposed GMRES failed in the adjoint sweep");
      const int nb = launch_adjoint_grad(p->md, p->P, uk, T.lam, T.dt, grad_g, T.partials, st);
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

}  // extern "C"
