// HIP kernels of libseird for gfx950 (wave64).
//
// Assembly is node-gather: one thread owns one node row and walks that
// node's element incidence records, so every output is written by exactly
// one thread (no atomics, no colour passes, deterministic).  The Jacobian
// is stored as a node-block matrix whose off-diagonal blocks are
// diagonal-plus-rank-one (10 values), which the SpMV exploits.
// Reductions use a fixed grid and a fixed combination order, so results
// are bitwise reproducible run to run.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include "kernels.h"

#include <algorithm>
#include <mutex>
#include <vector>

namespace seird {

// ----------------------------------------------------------------------
// nodal reaction (Eqs. seird1-5 / vec_component2) and its Jacobian
// ----------------------------------------------------------------------
__device__ inline void reaction_at(const double u[5], const ParamsDev &P, double g, double R[5]) {
  const double s = u[0], e = u[1], i = u[2], r = u[3], d = u[4];
  const double N = s + e + i + r + d;
  const double a = 1.0 - P.A / N;
  const double inf = a * g * (P.bI * i + P.bE * e) * s;
  R[0] = P.alpha * N - inf - P.mu * s;
  R[1] = inf - (P.sigma + P.gE + P.mu) * e;
  R[2] = P.sigma * e - (P.gR + P.gD + P.mu) * i;
  R[3] = P.gE * e + P.gR * i - P.mu * r;
  R[4] = P.gD * i;
}

// JR[c][c'] = d R_c / d u_c'
__device__ inline void reaction_jac_at(const double u[5], const ParamsDev &P, double g, double JR[5][5]) {
  const double s = u[0], e = u[1], i = u[2];
  const double N = u[0] + u[1] + u[2] + u[3] + u[4];
  const double a = 1.0 - P.A / N;
  const double dadN = P.A / (N * N);
  const double lam = g * (P.bI * i + P.bE * e);
  // d(a lam s)/du_c' = dadN lam s + a s dlam/du_c' + a lam [c'==S]
  double q[5];
  const double base = dadN * lam * s;
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = base;
  q[0] += a * lam;
  q[1] += a * s * g * P.bE;
  q[2] += a * s * g * P.bI;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    JR[0][c] = P.alpha - q[c];
    JR[1][c] = q[c];
    JR[2][c] = 0.0;
    JR[3][c] = 0.0;
    JR[4][c] = 0.0;
  }
  JR[0][0] -= P.mu;
  JR[1][1] -= P.sigma + P.gE + P.mu;
  JR[2][1] = P.sigma;
  JR[2][2] = -(P.gR + P.gD + P.mu);
  JR[3][1] = P.gE;
  JR[3][2] = P.gR;
  JR[3][3] = -P.mu;
  JR[4][2] = P.gD;
}

__device__ inline void load5(const double *p, double v[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) v[c] = p[c];
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// Node-indexed kernels remap the hardware block index so that every XCD
// gets one contiguous range of node blocks: neighbouring nodes (whose
// values the gathers share) then meet in the same L2.  A bijection on
// [0, nb) whatever the dispatch order.
constexpr int N_XCD = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b % N_XCD, idx = b / N_XCD;
  const int64_t per = nb / N_XCD, rem = nb % N_XCD;
  return x * per + (x < rem ? x : rem) + idx;
}
__device__ inline int64_t xcd_thread() {
  return xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

// ----------------------------------------------------------------------
// residual: one thread per node
// ----------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_residual(MeshDev m, ParamsDev P0, const double *__restrict__ gfield,
                                                  const double *__restrict__ u, const double *__restrict__ up,
                                                  double dt, const double *__restrict__ src, double *__restrict__ F) {
  const int64_t i = xcd_thread();
  if (i >= m.n) return;
  const ParamsDev P = m.inst ? m.Pinst[m.inst[i]] : P0;
  double ui[5];
  load5(u + 5 * i, ui);
  const double Ni = ui[0] + ui[1] + ui[2] + ui[3] + ui[4];
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t k = m.inc_ptr[i]; k < m.inc_ptr[i + 1]; ++k) {
    const int32_t j = m.inc_j[k], l = m.inc_l[k];
    const double Kii = m.inc_K[3 * k], Kij = m.inc_K[3 * k + 1], Kil = m.inc_K[3 * k + 2];
    double uj[5], ul[5];
    load5(u + 5 * (int64_t)j, uj);
    load5(u + 5 * (int64_t)l, ul);
    const double Nbar = (Ni + (uj[0] + uj[1] + uj[2] + uj[3] + uj[4]) + (ul[0] + ul[1] + ul[2] + ul[3] + ul[4])) *
                        (1.0 / 3.0);
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] += Nbar * (Kii * ui[c] + Kij * uj[c] + Kil * ul[c]);
  }
  const double g = gfield ? gfield[i] : 1.0;
  double R[5];
  reaction_at(ui, P, g, R);
  const double mi = m.mass[i];
  // time-derivative term: lumped m_i (u - u^n)_i, or consistent
  // sum_j M_ij (u - u^n)_j over the node and its graph neighbours
  double mt[5];
  if (m.cmass_d) {
    const double md = m.cmass_d[i];
#pragma unroll
    for (int c = 0; c < 5; ++c) mt[c] = md * (ui[c] - up[5 * i + c]);
    for (int64_t s = m.rowptr[i]; s < m.rowptr[i + 1]; ++s) {
      const int64_t j = m.col[s];
      const double mo = m.cmass_o[s];
#pragma unroll
      for (int c = 0; c < 5; ++c) mt[c] += mo * (u[5 * j + c] - up[5 * j + c]);
    }
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c) mt[c] = mi * (ui[c] - up[5 * i + c]);
  }
  // boundary flux of Eq. weakform: int (q . n) phi_i over the boundary
  // edges at node i, q P1 along the edge: (2 q_i + q_j) . n L / 6
  double bq[5] = {0, 0, 0, 0, 0};
  if (m.qflux) {
    for (int64_t b = m.bnd_ptr[i]; b < m.bnd_ptr[i + 1]; ++b) {
      const int64_t j = m.bnd_j[b];
      const double nx = m.bnd_nl[2 * b], ny = m.bnd_nl[2 * b + 1];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const double *qi = m.qflux + 10 * i + 2 * c, *qj = m.qflux + 10 * j + 2 * c;
        bq[c] += (2.0 * (qi[0] * nx + qi[1] * ny) + (qj[0] * nx + qj[1] * ny)) * (1.0 / 6.0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    double f = mt[c] + dt * P.nu[c] * acc[c] - dt * mi * R[c] - dt * bq[c];
    if (src) f -= dt * mi * src[5 * i + c];
    F[5 * i + c] = f;
  }
}

// ----------------------------------------------------------------------
// Jacobian.
//   diag[i][c][c'] = m_i (delta - dt dR_c/du_c') + dt nu_c (sum_T Nbar K_ii) delta
//                    + dt nu_c (1/3) sum_T sum_k K_ik u_c,k
//   off[s] = (a[5], b[5]): a_c = dt nu_c sum_T Nbar K_ij ; b_c = dt nu_c (1/3) sum_T sum_k K_ik u_c,k
// Two kernels: one thread per node row for the diagonal blocks, one thread
// per off-diagonal slot for the slots (each slot reads only the one or two
// elements holding its edge and writes its 10 values next to its
// neighbours' in memory).
// ----------------------------------------------------------------------
// element k's coupling of node i (state ui, total Ni) with its other two
// vertices j, l: Nbar and G3_c = dt nu_c (Kii u_c,i + Kij u_c,j + Kil u_c,l) / 3
__device__ inline void jac_element(const MeshDev &m, const double *__restrict__ u, const double (&ui)[5], double Ni,
                                   const double (&coef)[5], int64_t k, double &Nbar, double (&G3)[5]) {
  const int32_t j = m.inc_j[k], l = m.inc_l[k];
  const double Kii = m.inc_K[3 * k], Kij = m.inc_K[3 * k + 1], Kil = m.inc_K[3 * k + 2];
  double uj[5], ul[5];
  load5(u + 5 * (int64_t)j, uj);
  load5(u + 5 * (int64_t)l, ul);
  Nbar = (Ni + (uj[0] + uj[1] + uj[2] + uj[3] + uj[4]) + (ul[0] + ul[1] + ul[2] + ul[3] + ul[4])) * (1.0 / 3.0);
#pragma unroll
  for (int c = 0; c < 5; ++c) G3[c] = coef[c] * (Kii * ui[c] + Kij * uj[c] + Kil * ul[c]) * (1.0 / 3.0);
}

// diagonal blocks from the assembled stiffness, one thread per node row:
//   sum_T (K^T u_c)_i      = K_ii u_c,i + sum_s K_is u_c,col(s)
//   sum_T Nbar_T K^T_ii    = (N_i K_ii + sum_s W_s N_col(s)) / 3
// (W_s: K^T_ii summed over the elements holding the slot's edge), so the
// row reads each neighbour's state once instead of once per element
__global__ __launch_bounds__(256) void k_jacobian(MeshDev m, ParamsDev P0, const double *__restrict__ gfield,
                                                  const double *__restrict__ u, double dt, double *__restrict__ diag) {
  const int64_t i = xcd_thread();
  if (i >= m.n) return;
  const ParamsDev P = m.inst ? m.Pinst[m.inst[i]] : P0;
  double ui[5];
  load5(u + 5 * i, ui);
  const double Ni = ui[0] + ui[1] + ui[2] + ui[3] + ui[4];
  const double kii = m.kd[i];
  double ku[5], nk = Ni * kii;
#pragma unroll
  for (int c = 0; c < 5; ++c) ku[c] = kii * ui[c];
  for (int64_t s = m.rowptr[i]; s < m.rowptr[i + 1]; ++s) {
    double uj[5];
    load5(u + 5 * (int64_t)m.col[s], uj);
    const double ko = m.ko[s];
    nk += m.kw[s] * (uj[0] + uj[1] + uj[2] + uj[3] + uj[4]);
#pragma unroll
    for (int c = 0; c < 5; ++c) ku[c] += ko * uj[c];
  }
  const double g = gfield ? gfield[i] : 1.0;
  double JR[5][5];
  reaction_jac_at(ui, P, g, JR);
  const double mi = m.mass[i];
  const double mdiag = m.cmass_d ? m.cmass_d[i] : mi;  // the time-derivative term's diagonal
  double *D = diag + 25 * i;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double coef = dt * P.nu[c];
    const double da = coef * nk * (1.0 / 3.0), db = coef * ku[c] * (1.0 / 3.0);
#pragma unroll
    for (int cp = 0; cp < 5; ++cp) D[5 * c + cp] = -dt * mi * JR[c][cp] + db + (c == cp ? mdiag + da : 0.0);
  }
}

// off-diagonal slot s of row i: its 10 values summed over the elements
// that share the edge, in incidence-record order
__global__ __launch_bounds__(256) void k_jacobian_off(MeshDev m, ParamsDev P0, const double *__restrict__ u, double dt,
                                                      double *__restrict__ off) {
  const int64_t s = xcd_thread();
  if (s >= m.nslots) return;
  const int64_t i = m.slot_row[s];
  const int32_t e0 = m.slot_ek[2 * s], e1 = m.slot_ek[2 * s + 1];
  const ParamsDev P = m.inst ? m.Pinst[m.inst[i]] : P0;
  double ui[5];
  load5(u + 5 * i, ui);
  const double Ni = ui[0] + ui[1] + ui[2] + ui[3] + ui[4];
  double coef[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) coef[c] = dt * P.nu[c];
  double o[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int32_t ek = t == 0 ? e0 : e1;
    if (ek < 0) continue;
    const int64_t k = ek >> 1;
    double Nbar, G3[5];
    jac_element(m, u, ui, Ni, coef, k, Nbar, G3);
    const double Kx = m.inc_K[3 * k + 1 + (ek & 1)];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      o[c] += coef[c] * Nbar * Kx;
      o[5 + c] += G3[c];
    }
  }
  if (m.cmass_o) {
    const double mo = m.cmass_o[s];
#pragma unroll
    for (int c = 0; c < 5; ++c) o[c] += mo;
  }
#pragma unroll
  for (int q = 0; q < 10; ++q) off[10 * s + q] = o[q];
}

// ----------------------------------------------------------------------
// SpMV with the node-block Jacobian: y = J x, or y = b - J x when b != 0.
// Five lanes per node, lane c producing row c of the node's block row (of
// block column c for J^T): consecutive lanes then read consecutive matrix
// entries and write consecutive outputs.  Each output sums its terms in the
// order diagonal block, then slots in CSR order.
// ----------------------------------------------------------------------
constexpr int SPMV_WAVE_NODES = 12;  // nodes per wave (lanes 60..63 idle)

// A wave holds 12 whole nodes, so the five lanes of a node exchange their
// neighbour components with shuffles (each lane loads one).  The first
// SPMV_PF slots of a row are loaded before any of them is used (column
// indices, then neighbour values and matrix entries), so a wave has all of
// its row's loads in flight at once instead of one slot's chain at a time;
// the loads past the row's last slot re-read that slot (every node of a
// valid mesh has neighbours) and their terms are dropped, which keeps the
// loads unconditional.  Rows with more slots finish in a loop.
#ifndef SEIRD_SPMV_PF
#define SEIRD_SPMV_PF 6
#endif
constexpr int SPMV_PF = SEIRD_SPMV_PF;
__global__ __launch_bounds__(256) void k_spmv(MeshDev m, const double *__restrict__ diag,
                                              const double *__restrict__ off, const double *__restrict__ x,
                                              const double *__restrict__ b, double *__restrict__ y) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane % 5, g0 = lane - c;  // first lane of this node's group
  const int64_t i = (xcd_block(blockIdx.x, gridDim.x) * 4 + w) * SPMV_WAVE_NODES + lane / 5;
  if (lane >= 5 * SPMV_WAVE_NODES || i >= m.n) return;
  const int64_t s0 = m.rowptr[i], s1 = m.rowptr[i + 1];
  const int64_t slast = s1 > s0 ? s1 - 1 : s0;
  int32_t cj[SPMV_PF];
#pragma unroll
  for (int k = 0; k < SPMV_PF; ++k) cj[k] = m.col[min(s0 + k, slast)];
  // the node's own state: one load per lane, shared by shuffles
  const double xic = x[5 * i + c];
  double xi[5];
#pragma unroll
  for (int cp = 0; cp < 5; ++cp) xi[cp] = __shfl(xic, g0 + cp, 64);
  const double *D = diag + 25 * i + 5 * c;
  double dv[5];
#pragma unroll
  for (int cp = 0; cp < 5; ++cp) dv[cp] = D[cp];
  double xa[SPMV_PF], oa[SPMV_PF], ob[SPMV_PF];
#pragma unroll
  for (int k = 0; k < SPMV_PF; ++k) {
    const double *o = off + 10 * min(s0 + k, slast);
    xa[k] = x[5 * (int64_t)cj[k] + c];
    oa[k] = o[c];
    ob[k] = o[5 + c];
  }
  double acc = 0.0;
#pragma unroll
  for (int cp = 0; cp < 5; ++cp) acc += dv[cp] * xi[cp];
#pragma unroll
  for (int k = 0; k < SPMV_PF; ++k) {
    const double xjc = xa[k];
    const double S = __shfl(xjc, g0, 64) + __shfl(xjc, g0 + 1, 64) + __shfl(xjc, g0 + 2, 64) +
                     __shfl(xjc, g0 + 3, 64) + __shfl(xjc, g0 + 4, 64);
    if (s0 + k < s1) acc += oa[k] * xjc + ob[k] * S;
  }
  for (int64_t s = s0 + SPMV_PF; s < s1; ++s) {
    const double xjc = x[5 * (int64_t)m.col[s] + c];
    const double S = __shfl(xjc, g0, 64) + __shfl(xjc, g0 + 1, 64) + __shfl(xjc, g0 + 2, 64) +
                     __shfl(xjc, g0 + 3, 64) + __shfl(xjc, g0 + 4, 64);
    const double *o = off + 10 * s;
    acc += o[c] * xjc + o[5 + c] * S;
  }
  y[5 * i + c] = b ? b[5 * i + c] - acc : acc;
}

// y = J^T x (or b - J^T x): column j of J gathered through the transposed
// slots, with the same lane layout; lane c' of node j loads component c' of
// the neighbour's x, and the five lanes share their products for the
// rank-one term b . x_i.
__global__ __launch_bounds__(256) void k_spmv_t(MeshDev m, const double *__restrict__ diag,
                                                const double *__restrict__ off, const double *__restrict__ x,
                                                const double *__restrict__ b, double *__restrict__ y) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cp = lane % 5, g0 = lane - cp;  // first lane of this node's group
  const int64_t j = (xcd_block(blockIdx.x, gridDim.x) * 4 + w) * SPMV_WAVE_NODES + lane / 5;
  if (lane >= 5 * SPMV_WAVE_NODES || j >= m.n) return;
  const int64_t s0 = m.rowptr[j], s1 = m.rowptr[j + 1];
  int32_t ci[SPMV_PF], ts[SPMV_PF];
#pragma unroll
  for (int k = 0; k < SPMV_PF; ++k) {
    const bool v = s0 + k < s1;
    ci[k] = v ? m.col[s0 + k] : (int32_t)j;
    ts[k] = v ? m.tslot[s0 + k] : 0;
  }
  double xj[5];
  load5(x + 5 * j, xj);
  const double *D = diag + 25 * j + cp;
  double dv[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) dv[c] = D[5 * c];
  double xa[SPMV_PF], oa[SPMV_PF], ob[SPMV_PF];
#pragma unroll
  for (int k = 0; k < SPMV_PF; ++k) {
    const bool v = s0 + k < s1;
    const double *o = off + 10 * (int64_t)ts[k];
    xa[k] = x[5 * (int64_t)ci[k] + cp];
    oa[k] = v ? o[cp] : 0.0;
    ob[k] = v ? o[5 + cp] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 5; ++c) acc += dv[c] * xj[c];
#pragma unroll
  for (int k = 0; k < SPMV_PF; ++k) {
    const double xic = xa[k];
    const double pr = ob[k] * xic;
    const double bsum = __shfl(pr, g0, 64) + __shfl(pr, g0 + 1, 64) + __shfl(pr, g0 + 2, 64) +
                        __shfl(pr, g0 + 3, 64) + __shfl(pr, g0 + 4, 64);
    if (s0 + k < s1) acc += oa[k] * xic + bsum;
  }
  for (int64_t s = s0 + SPMV_PF; s < s1; ++s) {
    const double xic = x[5 * (int64_t)m.col[s] + cp];
    const double *o = off + 10 * (int64_t)m.tslot[s];  // block (i, j) lives at slot tslot of row i
    const double pr = o[5 + cp] * xic;
    const double bsum = __shfl(pr, g0, 64) + __shfl(pr, g0 + 1, 64) + __shfl(pr, g0 + 2, 64) +
                        __shfl(pr, g0 + 3, 64) + __shfl(pr, g0 + 4, 64);
    acc += o[cp] * xic + bsum;
  }
  y[5 * j + cp] = b ? b[5 * j + cp] - acc : acc;
}

// ----------------------------------------------------------------------
// deterministic reductions
// ----------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block of 256 threads -> one value (valid in thread 0)
__device__ inline double block_sum(double v, double *lds4) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds4[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
  return r;
}

// partials[k * nb + block] = sum over the block's indices of V_k . w
// (V_k = V + k*ldv, k < nv); if with_self, partials[nv*nb + b] = w . w.
template <int NVMAX>
__global__ __launch_bounds__(256) void k_mdot(const double *__restrict__ V, int64_t ldv, int nv,
                                              const double *__restrict__ w, int64_t N, int with_self,
                                              double *__restrict__ partials) {
  __shared__ double lds4[4];
  double acc[NVMAX + 1];
#pragma unroll
  for (int k = 0; k <= NVMAX; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride) {
    const double wv = w[idx];
#pragma unroll
    for (int k = 0; k < NVMAX; ++k)
      if (k < nv) acc[k] += V[k * ldv + idx] * wv;
    acc[NVMAX] += wv * wv;
  }
  const int nb = gridDim.x;
#pragma unroll
  for (int k = 0; k < NVMAX; ++k) {
    if (k < nv) {  // uniform over the block
      double r = block_sum(acc[k], lds4);
      if (threadIdx.x == 0) partials[(int64_t)k * nb + blockIdx.x] = r;
    }
  }
  if (with_self) {
    double r = block_sum(acc[NVMAX], lds4);
    if (threadIdx.x == 0) partials[(int64_t)nv * nb + blockIdx.x] = r;
  }
}

// out[k] = sum_b partials[k*nb + b] (fixed order), one block per k
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ partials, int nb,
                                                         double *__restrict__ out) {
  __shared__ double lds4[4];
  const int k = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) v += partials[(int64_t)k * nb + b];
  double r = block_sum(v, lds4);
  if (threadIdx.x == 0) out[k] = r;
}

// w -= sum_k h[k] V_k ; partial ||w||^2
template <int NVMAX>
__global__ __launch_bounds__(256) void k_maxpy_norm(double *__restrict__ w, const double *__restrict__ V, int64_t ldv,
                                                    const double *__restrict__ h, int nv, int64_t N,
                                                    double *__restrict__ partials) {
  __shared__ double lds4[4];
  __shared__ double hs[NVMAX];
  if (threadIdx.x < NVMAX) hs[threadIdx.x] = threadIdx.x < nv ? h[threadIdx.x] : 0.0;
  __syncthreads();
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride) {
    double v = w[idx];
#pragma unroll
    for (int k = 0; k < NVMAX; ++k)
      if (k < nv) v -= hs[k] * V[k * ldv + idx];
    w[idx] = v;
    acc += v * v;
  }
  double r = block_sum(acc, lds4);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// x += sum_k y[k] Z_k
template <int NVMAX>
__global__ __launch_bounds__(256) void k_gemv_update(double *__restrict__ x, const double *__restrict__ Z, int64_t ldz,
                                                     const double *__restrict__ y, int nv, int64_t N) {
  __shared__ double ys[NVMAX];
  if (threadIdx.x < NVMAX) ys[threadIdx.x] = threadIdx.x < nv ? y[threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride) {
    double v = x[idx];
#pragma unroll
    for (int k = 0; k < NVMAX; ++k)
      if (k < nv) v += ys[k] * Z[k * ldz + idx];
    x[idx] = v;
  }
}

// y = a*x (+ b*y if accumulate) ; alpha read from device memory when aptr
__global__ void k_axpby(double *__restrict__ y, const double *__restrict__ x, double a, const double *__restrict__ aptr,
                        int ainv, double b, int64_t N) {
  double aa = aptr ? (ainv ? 1.0 / aptr[0] : aptr[0]) : a;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride)
    y[idx] = aa * x[idx] + (b != 0.0 ? b * y[idx] : 0.0);
}

// y[0..N) = v for int arrays (queue counters)
__global__ void k_fill_int(int *__restrict__ y, int v, int N) {
  for (int idx = threadIdx.x; idx < N; idx += blockDim.x) y[idx] = v;
}

// y[0..N) = v (a fill kernel rather than a memset, so that it can sit in a
// captured stream)
__global__ void k_fill(double *__restrict__ y, double v, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride) y[idx] = v;
}

// ||F||^2 partials plus a nonfinite flag
__global__ __launch_bounds__(256) void k_norm2_partials(const double *__restrict__ x, const double *__restrict__ scale,
                                                        int64_t N, double *__restrict__ partials) {
  __shared__ double lds4[4];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride) {
    double v = x[idx];
    if (scale) v *= scale[idx / 5];
    acc += v * v;
  }
  double r = block_sum(acc, lds4);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// state check: count of nodes with N <= 0 or any nonfinite entry
// flags[instance of node]: bit 0 nonfinite entry, bit 1 total density <= 0
__global__ __launch_bounds__(256) void k_check_state(const double *__restrict__ u, int64_t n,
                                                     const int32_t *__restrict__ inst, int *__restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (inst) flags += inst[i];
  double v[5];
  load5(u + 5 * i, v);
  const double N = v[0] + v[1] + v[2] + v[3] + v[4];
  bool bad_nf = false;
#pragma unroll
  for (int c = 0; c < 5; ++c) bad_nf |= !isfinite(v[c]);
  if (bad_nf) atomicOr(flags, 1);
  else if (!(N > 0.0)) atomicOr(flags, 2);
}

// ----------------------------------------------------------------------
// Scalar CSR values of the node-block Jacobian: row 5 i + c lists, for the
// nodes j of {i} and its neighbours in increasing order, the five columns
// 5 j .. 5 j + 4 (the block (i, j) row c).  One thread per scalar row.
// ----------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_csr_values(MeshDev m, const double *__restrict__ diag,
                                                    const double *__restrict__ off,
                                                    const int64_t *__restrict__ csr_rowptr,
                                                    double *__restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 5 * m.n) return;
  const int64_t i = r / 5;
  const int c = (int)(r % 5);
  double *o = out + csr_rowptr[r];
  bool diag_done = false;
  auto put_diag = [&]() {
#pragma unroll
    for (int cp = 0; cp < 5; ++cp) o[cp] = diag[25 * i + 5 * c + cp];
    o += 5;
    diag_done = true;
  };
  for (int64_t s = m.rowptr[i]; s < m.rowptr[i + 1]; ++s) {
    if (!diag_done && m.col[s] > i) put_diag();
    const double a = off[10 * s + c], b = off[10 * s + 5 + c];
#pragma unroll
    for (int cp = 0; cp < 5; ++cp) o[cp] = b + (cp == c ? a : 0.0);
    o += 5;
  }
  if (!diag_done) put_diag();
}

// ----------------------------------------------------------------------
// Decoupled Picard-Gauss-Seidel sweep (Appendix A, Eq. weak_vec_implicit):
// the compartments are solved one after the other as scalar systems whose
// diffusion coefficient N and Allee factor a = 1 - A/N are lagged at the
// sweep's start (uk) while the compartments already updated in the sweep
// enter with their new values.  Compartment c's system is
//   A_c = diag(m_i (1 + dt q_c,i)) + dt nu_c Ksc(N^k),
//   rhs_c = m (u^n_c + dt f_c),
// with Ksc the scalar P1 stiffness weighted by the element-mean lagged
// density, q_c the loss rate of compartment c and f_c its gain:
//   S: q = a g (bI i + bE e) + mu,        f = alpha N^k
//   E: q = sigma + gE + mu - a g bE s,    f = a g bI s i
//   I: q = gR + gD + mu,                  f = sigma e
//   R: q = mu,                            f = gE e + gR i
//   D: q = 0,                             f = gD i
// (s, e, i from the current state; at the fixed point every lagged value
// equals the new one and u solves the coupled residual).
// ----------------------------------------------------------------------
// Ksc: Kd[i] = sum_{T ni i} Nbar_T K^T_ii, Ko[s] = sum over the triangles of
// edge (i, j) of Nbar_T K^T_ij (slot s = (i, j) of the node graph), each
// entry written once by the thread of node i.
constexpr int PGS_MAXINC = 16;  // element means held in registers per node
__global__ __launch_bounds__(256) void k_pgs_stiffness(MeshDev m, const double *__restrict__ uk,
                                                       double *__restrict__ Kd, double *__restrict__ Ko) {
  const int64_t i = xcd_thread();
  if (i >= m.n) return;
  double ui[5];
  load5(uk + 5 * i, ui);
  const double Ni = ui[0] + ui[1] + ui[2] + ui[3] + ui[4];
  const int64_t k0 = m.inc_ptr[i], k1 = m.inc_ptr[i + 1];
  auto nbar = [&](int64_t k) {
    double uj[5], ul[5];
    load5(uk + 5 * (int64_t)m.inc_j[k], uj);
    load5(uk + 5 * (int64_t)m.inc_l[k], ul);
    return (Ni + (uj[0] + uj[1] + uj[2] + uj[3] + uj[4]) + (ul[0] + ul[1] + ul[2] + ul[3] + ul[4])) * (1.0 / 3.0);
  };
  double nb[PGS_MAXINC];
  double kd = 0.0;
  for (int64_t k = k0; k < k1; ++k) {
    const double b = nbar(k);
    if (k - k0 < PGS_MAXINC) nb[k - k0] = b;
    kd += b * m.inc_K[3 * k];
  }
  Kd[i] = kd;
  for (int64_t s = m.rowptr[i]; s < m.rowptr[i + 1]; ++s) {
    double o = 0.0;
    for (int64_t k = k0; k < k1; ++k) {
      const bool atj = m.inc_sj[k] == s, atl = m.inc_sl[k] == s;
      if (!atj && !atl) continue;
      const double b = k - k0 < PGS_MAXINC ? nb[k - k0] : nbar(k);
      o += b * (atj ? m.inc_K[3 * k + 1] : m.inc_K[3 * k + 2]);
    }
    Ko[s] = o;
  }
}

// Compartment c's system: sdiag, soff (slot values) and, in correction
// form, r = rhs_c - A_c u_c (the update solves A_c delta = r).
__global__ __launch_bounds__(256) void k_pgs_system(MeshDev m, ParamsDev P, const double *__restrict__ gfield,
                                                    int c, double dt, const double *__restrict__ u,
                                                    const double *__restrict__ uk, const double *__restrict__ un,
                                                    const double *__restrict__ Kd, const double *__restrict__ Ko,
                                                    double *__restrict__ sdiag, double *__restrict__ soff,
                                                    double *__restrict__ r) {
  const int64_t i = xcd_thread();
  if (i >= m.n) return;
  double v[5], w[5];
  load5(u + 5 * i, v);
  load5(uk + 5 * i, w);
  const double Nk = w[0] + w[1] + w[2] + w[3] + w[4];
  const double a = 1.0 - P.A / Nk;
  const double g = gfield ? gfield[i] : 1.0;
  const double s = v[0], e = v[1], ii = v[2];
  double q, f;
  switch (c) {
    case 0: q = a * g * (P.bI * ii + P.bE * e) + P.mu; f = P.alpha * Nk; break;
    case 1: q = P.sigma + P.gE + P.mu - a * g * P.bE * s; f = a * g * P.bI * s * ii; break;
    case 2: q = P.gR + P.gD + P.mu; f = P.sigma * e; break;
    case 3: q = P.mu; f = P.gE * e + P.gR * ii; break;
    default: q = 0.0; f = P.gD * ii; break;
  }
  const double mi = m.mass[i];
  const double sc = dt * P.nu[c];
  // time-derivative term: lumped m_i, or the consistent mass row (the
  // reaction keeps nodal quadrature); boundary flux on the right-hand side
  const double md = m.cmass_d ? m.cmass_d[i] : mi;
  const double di = md + dt * mi * q + sc * Kd[i];
  sdiag[i] = di;
  double Au = di * v[c], Mun = md * un[5 * i + c];
  for (int64_t t = m.rowptr[i]; t < m.rowptr[i + 1]; ++t) {
    const int64_t j = m.col[t];
    const double mo = m.cmass_o ? m.cmass_o[t] : 0.0;
    const double o = mo + sc * Ko[t];
    soff[t] = o;
    Au += o * u[5 * j + c];
    Mun += mo * un[5 * j + c];
  }
  double bq = 0.0;
  if (m.qflux) {
    for (int64_t b = m.bnd_ptr[i]; b < m.bnd_ptr[i + 1]; ++b) {
      const int64_t j = m.bnd_j[b];
      const double nx = m.bnd_nl[2 * b], ny = m.bnd_nl[2 * b + 1];
      const double *qi = m.qflux + 10 * i + 2 * c, *qj = m.qflux + 10 * j + 2 * c;
      bq += (2.0 * (qi[0] * nx + qi[1] * ny) + (qj[0] * nx + qj[1] * ny)) * (1.0 / 6.0);
    }
  }
  r[i] = Mun + dt * mi * f + dt * bq - Au;
}

// y = A x (b == nullptr) or y = b - A x for a scalar matrix on the node
// graph (diagonal + one value per slot); one thread per row, terms summed
// diagonal first, then slots in order.
__global__ __launch_bounds__(256) void k_scalar_spmv(MeshDev m, const double *__restrict__ sdiag,
                                                     const double *__restrict__ soff, const double *__restrict__ x,
                                                     const double *__restrict__ b, double *__restrict__ y) {
  const int64_t i = xcd_thread();
  if (i >= m.n) return;
  double acc = sdiag[i] * x[i];
  for (int64_t t = m.rowptr[i]; t < m.rowptr[i + 1]; ++t) acc += soff[t] * x[m.col[t]];
  y[i] = b ? b[i] - acc : acc;
}

// u_c += delta (dinv == nullptr) or u_c += r / sdiag (a diagonal system)
__global__ __launch_bounds__(256) void k_pgs_update(double *__restrict__ u, int c, const double *__restrict__ delta,
                                                    const double *__restrict__ sdiag, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u[5 * i + c] += sdiag ? delta[i] / sdiag[i] : delta[i];
}

// ----------------------------------------------------------------------
// Segmented reductions.  A vector of N entries is split into segments (one
// per problem instance; a single problem is one segment).  Every segment is
// cut into chunks of SEG_CH entries, one block per chunk; block b sums its
// chunk (thread t: entries t, t+256, ...) and writes a partial; the partials
// of a segment are then summed by one block in a fixed order.  The result
// for a segment therefore does not depend on the other segments.
// ----------------------------------------------------------------------
struct SegView {
  const int64_t *seg_start;   // [S+1] entry offsets
  const int64_t *blk_start;   // [S+1] block offsets
  const int32_t *block_seg;   // [B] segment of each block
  const uint8_t *active;      // [S] (nullable: all active)
  int S, B;
};

SegView SegHost::view() const { return SegView{d_seg_start, d_blk_start, d_block_seg, d_active, S, B}; }

__device__ inline void seg_range(const SegView &v, int b, int &sg, int64_t &lo, int64_t &hi) {
  sg = v.block_seg[b];
  lo = v.seg_start[sg] + (int64_t)(b - v.blk_start[sg]) * SEG_CH;
  hi = min(lo + (int64_t)SEG_CH, v.seg_start[sg + 1]);
}

// partials[k * B + b] = chunk sum of V_k . w (k < nv); with_self: row nv = w . w
template <int NVMAX>
__global__ __launch_bounds__(256) void k_seg_mdot(SegView v, const double *__restrict__ V, int64_t ldv, int nv,
                                                  const double *__restrict__ w, int with_self,
                                                  double *__restrict__ partials) {
  __shared__ double lds4[4];
  int sg;
  int64_t lo, hi;
  seg_range(v, blockIdx.x, sg, lo, hi);
  double acc[NVMAX + 1];
#pragma unroll
  for (int k = 0; k <= NVMAX; ++k) acc[k] = 0.0;
  if (!v.active || v.active[sg]) {
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += 256) {
      const double wv = w[idx];
#pragma unroll
      for (int k = 0; k < NVMAX; ++k)
        if (k < nv) acc[k] += V[k * ldv + idx] * wv;
      acc[NVMAX] += wv * wv;
    }
  }
#pragma unroll
  for (int k = 0; k < NVMAX; ++k) {
    if (k < nv) {
      const double r = block_sum(acc[k], lds4);
      if (threadIdx.x == 0) partials[(int64_t)k * v.B + blockIdx.x] = r;
    }
  }
  if (with_self) {
    const double r = block_sum(acc[NVMAX], lds4);
    if (threadIdx.x == 0) partials[(int64_t)nv * v.B + blockIdx.x] = r;
  }
}

// out[sg * ldo + k] = sum of the partials of segment sg, row k (one block per (sg, k))
__global__ __launch_bounds__(256) void k_seg_reduce(SegView v, const double *__restrict__ partials, int nrows,
                                                    double *__restrict__ out, int ldo, int row_off) {
  __shared__ double lds4[4];
  const int sg = blockIdx.x / nrows, k = blockIdx.x % nrows;
  double a = 0.0;
  const int64_t b0 = v.blk_start[sg], b1 = v.blk_start[sg + 1];
  for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) a += partials[(int64_t)k * v.B + b];
  const double r = block_sum(a, lds4);
  if (threadIdx.x == 0) out[(int64_t)sg * ldo + row_off + k] = r;
}

// w -= sum_k h[sg][k] V_k on active segments; partial ||w||^2
template <int NVMAX>
__global__ __launch_bounds__(256) void k_seg_maxpy_norm(SegView v, double *__restrict__ w, const double *__restrict__ V,
                                                        int64_t ldv, const double *__restrict__ h, int ldh, int nv,
                                                        double *__restrict__ partials) {
  __shared__ double lds4[4];
  __shared__ double hs[NVMAX];
  int sg;
  int64_t lo, hi;
  seg_range(v, blockIdx.x, sg, lo, hi);
  const bool act = !v.active || v.active[sg];
  if (threadIdx.x < NVMAX) hs[threadIdx.x] = (act && threadIdx.x < nv) ? h[(int64_t)sg * ldh + threadIdx.x] : 0.0;
  __syncthreads();
  double acc = 0.0;
  if (act) {
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += 256) {
      double x = w[idx];
#pragma unroll
      for (int k = 0; k < NVMAX; ++k)
        if (k < nv) x -= hs[k] * V[k * ldv + idx];
      w[idx] = x;
      acc += x * x;
    }
  }
  const double r = block_sum(acc, lds4);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// x += sum_k y[sg][k] Z_k on active segments
template <int NVMAX>
__global__ __launch_bounds__(256) void k_seg_gemv_update(SegView v, double *__restrict__ x, const double *__restrict__ Z,
                                                         int64_t ldz, const double *__restrict__ y, int ldy, int nv) {
  __shared__ double ys[NVMAX];
  int sg;
  int64_t lo, hi;
  seg_range(v, blockIdx.x, sg, lo, hi);
  const bool act = !v.active || v.active[sg];
  if (threadIdx.x < NVMAX) ys[threadIdx.x] = (act && threadIdx.x < nv) ? y[(int64_t)sg * ldy + threadIdx.x] : 0.0;
  __syncthreads();
  if (!act) return;
  for (int64_t idx = lo + threadIdx.x; idx < hi; idx += 256) {
    double t = x[idx];
#pragma unroll
    for (int k = 0; k < NVMAX; ++k)
      if (k < nv) t += ys[k] * Z[k * ldz + idx];
    x[idx] = t;
  }
}

// y = a[sg] * x + b * y on active segments (a per segment, from device memory)
__global__ __launch_bounds__(256) void k_seg_axpby(SegView v, double *__restrict__ y, const double *__restrict__ x,
                                                   const double *__restrict__ a, double b) {
  int sg;
  int64_t lo, hi;
  seg_range(v, blockIdx.x, sg, lo, hi);
  if (v.active && !v.active[sg]) return;
  const double aa = a[sg];
  for (int64_t idx = lo + threadIdx.x; idx < hi; idx += 256) y[idx] = aa * x[idx] + (b != 0.0 ? b * y[idx] : 0.0);
}

// partial sum of (scale[idx/5] x[idx])^2 per block (scale nullable)
__global__ __launch_bounds__(256) void k_seg_norm2(SegView v, const double *__restrict__ x,
                                                   const double *__restrict__ scale, double *__restrict__ partials) {
  __shared__ double lds4[4];
  int sg;
  int64_t lo, hi;
  seg_range(v, blockIdx.x, sg, lo, hi);
  double acc = 0.0;
  for (int64_t idx = lo + threadIdx.x; idx < hi; idx += 256) {
    double t = x[idx];
    if (scale) t *= scale[idx / 5];
    acc += t * t;
  }
  const double r = block_sum(acc, lds4);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// ----------------------------------------------------------------------
// Tile storage (subdomain envelopes, coarse band): init, extraction of
// R_i A R_i^T, conversion
// ----------------------------------------------------------------------
// Tile addressing of one system's factor storage (envelope layout when the
// row table is given, else band layout; see SubInfo).
struct TileRows {
  int64_t base;
  int32_t nt, bl, bu;
  const int32_t *row, *lo;
  template <int T>
  __device__ inline int64_t at(int K, int J) const {  // entry offset of tile (K, J)
    return base + (row ? (int64_t)row[K] + (J - lo[K]) : (int64_t)K * (bl + bu + 1) + (J - K + bl)) * (T * T);
  }
  __device__ inline int first(int K) const { return row ? lo[K] : max(0, K - bl); }
  __device__ inline int last(int K) const { return row ? lo[K] + (row[K + 1] - row[K]) - 1 : min(nt - 1, K + bu); }
  // block row K at once: tile (K, J) starts at entry off0 + J T^2, for J
  // in first .. last (one read of the row tables instead of one per tile)
  template <int T>
  __device__ inline void row_info(int K, int64_t &off0, int &first_, int &last_) const {
    if (row) {
      const int r0 = row[K], r1 = row[K + 1], l0 = lo[K];
      off0 = base + ((int64_t)r0 - l0) * (T * T);
      first_ = l0;
      last_ = l0 + (r1 - r0) - 1;
    } else {
      off0 = base + ((int64_t)K * (bl + bu + 1) - K + bl) * (T * T);
      first_ = max(0, K - bl);
      last_ = min(nt - 1, K + bu);
    }
  }
};
__device__ inline TileRows tile_rows(const SubInfo &s, const int32_t *erow, const int32_t *elo) {
  TileRows r;
  r.base = s.base;
  r.nt = s.nt;
  r.bl = s.bl;
  r.bu = s.bu;
  r.row = s.env_off >= 0 ? erow + s.env_off : nullptr;
  r.lo = s.env_off >= 0 ? elo + s.env_off : nullptr;
  return r;
}
// entry (l, lp) of a system's matrix, or -1 when it lies outside the
// stored tiles
template <int T>
__device__ inline int64_t tile_entry_rows(const TileRows &R, int32_t l, int32_t lp) {
  const int32_t K = l / T, J = lp / T;
  if (l < 0 || lp < 0 || K >= R.nt || J < R.first(K) || J > R.last(K)) return -1;
  return R.at<T>(K, J) + (l % T) * T + (lp % T);
}

template <int T>
__device__ inline int64_t tile_entry(const SubInfo &s, int32_t l, int32_t lp) {
  const int32_t K = l / T, J = lp / T;
  const int32_t W = s.bl + s.bu + 1;
  return s.base + ((int64_t)K * W + (J - K + s.bl)) * (T * T) + (l % T) * T + (lp % T);
}

// same, returning -1 when (l, lp) falls outside the stored tile band
template <int T>
__device__ inline int64_t tile_entry_checked(const SubInfo &s, int32_t l, int32_t lp) {
  const int32_t K = l / T, J = lp / T;
  const int32_t slot = J - K + s.bl;
  if (l < 0 || lp < 0 || K >= s.nt || J >= s.nt || slot < 0 || slot > s.bl + s.bu) return -1;
  return tile_entry<T>(s, l, lp);
}

// identity on the padded diagonal of the last block row (storage zeroed before)
template <int T, class ET>
__global__ void k_pad_identity(ET *__restrict__ F, const SubInfo *__restrict__ subs, const int32_t *__restrict__ erow,
                               const int32_t *__restrict__ elo, int nsubs) {
  const int s = blockIdx.x;
  if (s >= nsubs) return;
  const SubInfo si = subs[s];
  const TileRows R = tile_rows(si, erow, elo);
  for (int32_t l = si.n_loc + threadIdx.x; l < si.nt * T; l += blockDim.x) F[tile_entry_rows<T>(R, l, l)] = (ET)1.0;
}

// Subdomain matrices A_i = R_i A R_i^T (Eq. RAS) written into the tile
// envelope.  One workgroup per subdomain tile row writes every stored entry
// of that row exactly once: the matrix entry, zero, or 1 on the padded
// diagonal, so the storage needs no clearing beforehand.  A thread owns one
// row of a tile and 4 consecutive columns; the nonzero node blocks of its
// row are the extraction entries of its local node.  BS = 5 (the coupled
// Jacobian): diagonal blocks from diag [n][25], off-diagonal block
// (c, c') = b_c + a_c [c = c'] from off [slots][10].  BS = 1 (one
// compartment's scalar matrix): diag [n] and off [slots].  DENSE (BS = 5,
// the Galerkin coarse matrix on the coarse graph): off-diagonal blocks
// dense, off [slots][25] row-major.
template <int T, class ET, int MAXE, int BS = 5, bool DENSE = false>
__global__ __launch_bounds__(256) void k_extract_tiles(ET *__restrict__ F, const SubInfo *__restrict__ subs,
                                                       const int32_t *__restrict__ trow_ptr,
                                                       const int32_t *__restrict__ trow_sub,
                                                       const int32_t *__restrict__ erow,
                                                       const int32_t *__restrict__ elo,
                                                       const ExtractEntry *__restrict__ ent,
                                                       const int32_t *__restrict__ ent_ptr,
                                                       const double *__restrict__ diag,
                                                       const double *__restrict__ off) {
  constexpr int CH = T / 4;          // 4-column chunks per tile row
  constexpr int PER = T * CH;        // threads per tile
  constexpr int TPP = 256 / PER;     // tiles per pass
  const int gK = blockIdx.x;
  const int s0 = trow_sub[gK];  // trow_ptr[s0] <= gK < trow_ptr[s0 + 1]
  const SubInfo si = subs[s0];
  const TileRows R = tile_rows(si, erow, elo);
  const int K = gK - trow_ptr[s0];
  const int tid = threadIdx.x, tt = tid / PER, a = (tid % PER) / CH, g = tid % CH;
  const int32_t l = K * T + a;  // local row
  const int32_t p = l / BS, c = l % BS;
  const bool real = l < si.n_loc;
  int32_t e0 = 0, e1 = 0;
  if (real) {
    const int64_t nb = si.l2g_off / BS + p;
    e0 = ent_ptr[nb];
    e1 = ent_ptr[nb + 1];
  }
  // the row's node blocks held in MAXE registers (column node, value
  // reference); nodes with more blocks search the entry list in memory
  const int32_t ne = e1 - e0;
  const bool inreg = ne <= MAXE;
  int32_t qv[MAXE], rv[MAXE], qlo = INT32_MAX, qhi = -1;
#pragma unroll
  for (int k = 0; k < MAXE; ++k) {
    const bool have = inreg && k < ne;
    qv[k] = have ? ent[e0 + k].q : -1;
    rv[k] = have ? ent[e0 + k].ref : 0;
    if (have) {
      qlo = min(qlo, qv[k]);
      qhi = max(qhi, qv[k]);
    }
  }
  auto value = [&](int32_t ref, int cp) -> double {
    if constexpr (BS == 1) {
      return ref < 0 ? diag[-(int64_t)ref - 1] : off[ref];
    } else {
      if (ref < 0) return diag[25 * (int64_t)(-ref - 1) + 5 * c + cp];
      if constexpr (DENSE) return off[25 * (int64_t)ref + 5 * c + cp];
      const double *o = off + 10 * (int64_t)ref;
      return o[5 + c] + (cp == c ? o[c] : 0.0);
    }
  };
  const int J1 = R.last(K);
  for (int J = R.first(K) + tt; J <= J1; J += TPP) {
    const int32_t lb0 = J * T + 4 * g;  // first column of the chunk
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (BS == 1) {
      // every column is its own node block: look each one up
      if (real && inreg) {
        if (lb0 + 3 >= qlo && lb0 <= qhi) {
#pragma unroll
          for (int k = 0; k < MAXE; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (qv[k] == lb0 + u) v[u] = value(rv[k], 0);
        }
      } else if (real) {
        for (int32_t k = e0; k < e1; ++k) {
          const int32_t d0 = ent[k].q - lb0;
          if (d0 >= 0 && d0 < 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (u == d0) v[u] = value(ent[k].ref, 0);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (lb0 + u == l) v[u] = 1.0;
      }
    } else if (real && inreg) {
      // columns lb0 .. lb0 + 3 belong to at most two node blocks qa, qb
      const int32_t qa = lb0 / 5, qb = (lb0 + 3) / 5;
      if (qb >= qlo && qa <= qhi) {
        int32_t ra = 0, rb = 0;
        bool ha = false, hb = false;
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          if (qv[k] == qa) {
            ha = true;
            ra = rv[k];
          }
          if (qv[k] == qb) {
            hb = true;
            rb = rv[k];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool inb = lb0 + u >= 5 * qb;
          if (inb ? hb : ha) v[u] = value(inb ? rb : ra, lb0 + u - 5 * (inb ? qb : qa));
        }
      }
    } else if (real) {
      for (int32_t k = e0; k < e1; ++k) {
        const int32_t d0 = lb0 - 5 * ent[k].q;  // chunk start relative to node block q
        if (d0 <= -4 || d0 >= 5) continue;
        const int32_t ref = ent[k].ref;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (d0 + u >= 0 && d0 + u < 5) v[u] = value(ref, d0 + u);
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (lb0 + u == l) v[u] = 1.0;
    }
    // non-temporal: the factorisation reads the tiles long after, so the
    // stores need not stay in the caches
    ET *dst = F + R.at<T>(K, J) + a * T + 4 * g;
    if constexpr (sizeof(ET) == 8) {
      typedef double d4 __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(d4{v[0], v[1], v[2], v[3]}, reinterpret_cast<d4 *>(dst));
    } else {
      typedef float f4 __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(f4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]}, reinterpret_cast<f4 *>(dst));
    }
  }
}

// Galerkin coarse matrix: coarse block k (local positions p, q) =
// sum_j w_j * fine block(ref_j).  One wave per coarse block: lanes stride
// over its contributions, each lane accumulates the 25 entries, then a
// fixed-order wave reduction leaves the block's entries in every lane.
// DENSE: the fine blocks are dense 5x5 (off [slots][25]) instead of the
// Jacobian's diag(a) + b 1^T form; gw null: every weight is 1.
template <bool DENSE = false>
__device__ inline void galerkin_sum(int64_t k, int lane, const int64_t *__restrict__ gptr,
                                    const int32_t *__restrict__ gref, const double *__restrict__ gw,
                                    const double *__restrict__ diag, const double *__restrict__ off,
                                    double (&acc)[25]) {
#pragma unroll
  for (int e = 0; e < 25; ++e) acc[e] = 0.0;
  for (int64_t j = gptr[k] + lane; j < gptr[k + 1]; j += 64) {
    const int32_t ref = gref[j];
    const double w = gw ? gw[j] : 1.0;
    if (ref < 0 || DENSE) {
      const double *D = ref < 0 ? diag + 25 * (int64_t)(-ref - 1) : off + 25 * (int64_t)ref;
#pragma unroll
      for (int e = 0; e < 25; ++e) acc[e] += w * D[e];
    } else {
      const double *o = off + 10 * (int64_t)ref;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const double b = w * o[5 + c];
#pragma unroll
        for (int cp = 0; cp < 5; ++cp) acc[5 * c + cp] += b;
        acc[5 * c + c] += w * o[c];
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 25; ++e) acc[e] = wave_sum(acc[e]);
}

// entry `lane` (< 25) of the reduced block
__device__ inline double galerkin_pick(const double (&acc)[25], int lane) {
  double v = 0.0;
#pragma unroll
  for (int e = 0; e < 25; ++e)
    if (e == lane) v = acc[e];
  return v;
}

// written into the coarse tile-band storage (direct coarse solve)
template <int T>
__global__ __launch_bounds__(256) void k_galerkin(double *__restrict__ F, SubInfo cs, const int32_t *__restrict__ gp,
                                                  const int32_t *__restrict__ gq, const int64_t *__restrict__ gptr,
                                                  const int32_t *__restrict__ gref, const double *__restrict__ gw,
                                                  int64_t nblk, const double *__restrict__ diag,
                                                  const double *__restrict__ off, int *status) {
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (k >= nblk) return;  // uniform per wave
  double acc[25];
  galerkin_sum(k, lane, gptr, gref, gw, diag, off, acc);
  if (lane < 25) {
    const double v = galerkin_pick(acc, lane);
    const int c = lane / 5, cp = lane % 5;
    const int64_t at = tile_entry_checked<T>(cs, 5 * gp[k] + c, 5 * gq[k] + cp);
    if (at < 0)
      atomicOr(status, 2);
    else
      F[at] = v;
  }
}

// written as node blocks of the coarse graph (Krylov coarse solve): block k
// goes to the diagonal block of position -dst-1 or to slot dst
template <bool DENSE>
__global__ __launch_bounds__(256) void k_galerkin_blocks(double *__restrict__ cdiag, double *__restrict__ coff,
                                                         const int32_t *__restrict__ gdst,
                                                         const int64_t *__restrict__ gptr,
                                                         const int32_t *__restrict__ gref,
                                                         const double *__restrict__ gw, int64_t nblk,
                                                         const double *__restrict__ diag,
                                                         const double *__restrict__ off) {
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (k >= nblk) return;  // uniform per wave
  double acc[25];
  galerkin_sum<DENSE>(k, lane, gptr, gref, gw, diag, off, acc);
  if (lane < 25) {
    const double v = galerkin_pick(acc, lane);
    const int32_t d = gdst[k];
    double *dst = d < 0 ? cdiag + 25 * (int64_t)(-d - 1) : coff + 25 * (int64_t)d;
    dst[lane] = v;
  }
}

// y = A x (or b - A x) for a matrix of dense 5x5 node blocks on a graph:
// diag [n][25], off [slots][25] (row-major blocks).  Five lanes per node,
// lane c producing row c; each output sums the diagonal block, then the
// slots in CSR order.
__global__ __launch_bounds__(256) void k_block_spmv(int64_t n, const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const double *__restrict__ diag,
                                                    const double *__restrict__ off, const double *__restrict__ x,
                                                    const double *__restrict__ b, double *__restrict__ y) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane % 5;
  const int64_t i = ((int64_t)blockIdx.x * 4 + w) * SPMV_WAVE_NODES + lane / 5;
  if (lane >= 5 * SPMV_WAVE_NODES || i >= n) return;
  double xi[5];
  load5(x + 5 * i, xi);
  const double *D = diag + 25 * i + 5 * c;
  double acc = 0.0;
#pragma unroll
  for (int cp = 0; cp < 5; ++cp) acc += D[cp] * xi[cp];
  for (int64_t s = rowptr[i]; s < rowptr[i + 1]; ++s) {
    double xj[5];
    load5(x + 5 * (int64_t)col[s], xj);
    const double *o = off + 25 * s + 5 * c;
#pragma unroll
    for (int cp = 0; cp < 5; ++cp) acc += o[cp] * xj[cp];
  }
  y[5 * i + c] = b ? b[5 * i + c] - acc : acc;
}

// ----------------------------------------------------------------------
// Aggregation AMG over dense 5x5 node blocks (V-cycle of the coarse solver)
// ----------------------------------------------------------------------
// dinv = inverse of every diagonal block (Gauss-Jordan with partial
// pivoting, one thread per node); *status |= 1 on a singular block
__global__ __launch_bounds__(256) void k_block_inv5(int64_t n, const double *__restrict__ diag,
                                                    double *__restrict__ dinv, int *status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a[5][5], x[5][5];
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      a[r][c] = diag[25 * i + 5 * r + c];
      x[r][c] = r == c ? 1.0 : 0.0;
    }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    int p = k;
    double best = fabs(a[k][k]);
#pragma unroll
    for (int r = k + 1; r < 5; ++r)
      if (fabs(a[r][k]) > best) {
        best = fabs(a[r][k]);
        p = r;
      }
    if (!(best > 0.0) || !isfinite(best)) {
      atomicOr(status, 1);
      return;
    }
    // swap rows k and p (selects, so the arrays stay in registers)
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double t0 = a[k][c], t1 = x[k][c];
#pragma unroll
      for (int r = k + 1; r < 5; ++r)
        if (r == p) {
          a[k][c] = a[r][c];
          a[r][c] = t0;
          x[k][c] = x[r][c];
          x[r][c] = t1;
        }
    }
    const double rp = 1.0 / a[k][k];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      a[k][c] *= rp;
      x[k][c] *= rp;
    }
#pragma unroll
    for (int r = 0; r < 5; ++r)
      if (r != k) {
        const double f = a[r][k];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          a[r][c] -= f * a[k][c];
          x[r][c] -= f * x[k][c];
        }
      }
  }
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int c = 0; c < 5; ++c) dinv[25 * i + 5 * r + c] = x[r][c];
}

// x += omega D^{-1} r over the node blocks (lane c of a node: row c)
__global__ __launch_bounds__(256) void k_block_jacobi(int64_t n, const double *__restrict__ dinv,
                                                      const double *__restrict__ r, double omega,
                                                      double *__restrict__ x) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 5 * n) return;
  const int64_t i = idx / 5;
  const int c = (int)(idx % 5);
  const double *D = dinv + 25 * i + 5 * c;
  double a = 0.0;
#pragma unroll
  for (int cp = 0; cp < 5; ++cp) a += D[cp] * r[5 * i + cp];
  x[idx] += omega * a;
}

// bc[a] = sum over the aggregate's member nodes (in list order) of r
__global__ __launch_bounds__(256) void k_agg_restrict(int64_t nagg, const int64_t *__restrict__ agg_ptr,
                                                      const int32_t *__restrict__ agg_nodes,
                                                      const double *__restrict__ r, double *__restrict__ bc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 5 * nagg) return;
  const int64_t a = idx / 5;
  const int c = (int)(idx % 5);
  double s = 0.0;
  for (int64_t k = agg_ptr[a]; k < agg_ptr[a + 1]; ++k) s += r[5 * (int64_t)agg_nodes[k] + c];
  bc[idx] = s;
}

// x[i] += xc[agg(i)] per component
__global__ __launch_bounds__(256) void k_agg_prolong(int64_t n, const int32_t *__restrict__ agg,
                                                     const double *__restrict__ xc, double *__restrict__ x) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 5 * n) return;
  const int64_t i = idx / 5;
  x[idx] += xc[5 * (int64_t)agg[i] + idx % 5];
}

// y = M b for a dense m x m matrix (row-major), one thread per row
__global__ __launch_bounds__(256) void k_dense_gemv(int m, const double *__restrict__ M, const double *__restrict__ b,
                                                    double *__restrict__ y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const double *row = M + (int64_t)r * m;
  double s = 0.0;
  for (int c = 0; c < m; ++c) s += row[c] * b[c];
  y[r] = s;
}

template <class FT>
__device__ inline FT to_ft(double v);
template <>
__device__ inline double to_ft<double>(double v) { return v; }
template <>
__device__ inline float to_ft<float>(double v) { return (float)v; }
template <>
__device__ inline __hip_bfloat16 to_ft<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }
template <class FT>
__device__ inline double from_ft(FT v);
template <>
__device__ inline double from_ft<double>(double v) { return v; }
template <>
__device__ inline double from_ft<float>(float v) { return (double)v; }
template <>
__device__ inline double from_ft<__hip_bfloat16>(__hip_bfloat16 v) { return (double)__bfloat162float(v); }

template <class FT, class ST>
__global__ void k_convert(FT *__restrict__ dst, const ST *__restrict__ src, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride)
    dst[idx] = to_ft<FT>((double)src[idx]);
}

// ----------------------------------------------------------------------
// Tile LU without pivoting (right-looking, block version; tile 16 and the
// coarse band).
// Device routines work on one tile operation with the whole workgroup
// (256 threads).  LDS tiles are padded to T+1 columns.
// ----------------------------------------------------------------------
template <int T, class CT = double>
struct LuLds {
  CT D[T][T + 1];   // diagonal tile being factored
  CT Li[T][T + 1];  // L_KK^{-1} (unit lower)
  CT Ui[T][T + 1];  // U_KK^{-1} (upper)
  CT S[T][T + 1];   // staging
};

// Factor the diagonal tile at dk in place and replace it by (strict lower of
// L^{-1}) + (upper of U^{-1}); keeps Li/Ui in LDS.  Raises *status on a bad pivot.
template <int T, class CT>
__device__ void lu_diag_tile(CT *__restrict__ dk, LuLds<T, CT> &L, int *status) {
  const int tid = threadIdx.x;
  for (int e = tid; e < T * T; e += 256) L.D[e / T][e % T] = dk[e];
  __syncthreads();
  for (int k = 0; k < T; ++k) {
    const CT piv = L.D[k][k];
    if (tid == 0 && (!isfinite((double)piv) || fabs((double)piv) < 1e-300)) atomicOr(status, 1);
    const CT rp = (CT)1 / piv;
    for (int i = k + 1 + tid; i < T; i += 256) L.D[i][k] *= rp;
    __syncthreads();
    const int w = T - k - 1;
    for (int e = tid; e < w * w; e += 256) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      L.D[i][j] -= L.D[i][k] * L.D[k][j];
    }
    __syncthreads();
  }
  // inverses: Li (forward over k), Ui (backward over k)
  for (int e = tid; e < T * T; e += 256) {
    const int i = e / T, j = e % T;
    L.Li[i][j] = (i == j) ? 1.0 : 0.0;
    L.Ui[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < T; ++k) {
    // Li: rows i > k, columns j <= k: Li[i][j] -= L[i][k] Li[k][j]
    // Ui: row kk = T-1-k is final after scaling by 1/U[kk][kk]
    const int kk = T - 1 - k;
    const CT ud = (CT)1 / L.D[kk][kk];
    for (int j = kk + tid; j < T; j += 256) L.Ui[kk][j] *= ud;
    __syncthreads();
    const int nl = (T - 1 - k) * (k + 1);
    for (int e = tid; e < nl; e += 256) {
      const int i = k + 1 + e / (k + 1), j = e % (k + 1);
      L.Li[i][j] -= L.D[i][k] * L.Li[k][j];
    }
    // Ui: rows i < kk, columns j >= kk
    const int nu = kk * (T - kk);
    for (int e = tid; e < nu; e += 256) {
      const int i = e / (T - kk), j = kk + e % (T - kk);
      L.Ui[i][j] -= L.D[i][kk] * L.Ui[kk][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < T * T; e += 256) {
    const int i = e / T, j = e % T;
    dk[e] = (i > j) ? L.Li[i][j] : L.Ui[i][j];
  }
  __syncthreads();
}

// load Li/Ui from a stored (inverted) diagonal tile
template <int T>
__device__ void load_diag_inverses(const double *__restrict__ dk, LuLds<T, double> &L) {
  for (int e = threadIdx.x; e < T * T; e += 256) {
    const int i = e / T, j = e % T;
    const double v = dk[e];
    L.Li[i][j] = (i > j) ? v : (i == j ? 1.0 : 0.0);
    L.Ui[i][j] = (i <= j) ? v : 0.0;
  }
  __syncthreads();
}

// X = A Ui (lower panel) or X = Li A (upper panel), in place at tile a
template <int T>
__device__ void panel_tile(double *__restrict__ a, LuLds<T, double> &L, bool lower) {
  for (int e = threadIdx.x; e < T * T; e += 256) L.S[e / T][e % T] = a[e];
  __syncthreads();
  for (int e = threadIdx.x; e < T * T; e += 256) {
    const int i = e / T, j = e % T;
    double acc = 0.0;
    if (lower) {
      for (int k = 0; k <= j; ++k) acc += L.S[i][k] * L.Ui[k][j];
    } else {
      for (int k = 0; k <= i; ++k) acc += L.Li[i][k] * L.S[k][j];
    }
    a[e] = acc;
  }
  __syncthreads();
}

// C -= A B  with A staged in Sa (LDS) and B in Sb (LDS), C in global
template <int T>
__device__ void schur_tile(double *__restrict__ C, const double (*Sa)[T + 1], const double (*Sb)[T + 1]) {
  constexpr int PER = (T * T) / 256;  // outputs per thread: 4 (T=32) or 1 (T=16)
  if constexpr (PER == 4) {
    // 2x2 register block per thread
    const int bi = (threadIdx.x / 16) * 2, bj = (threadIdx.x % 16) * 2;
    double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
#pragma unroll 8
    for (int k = 0; k < T; ++k) {
      const double a0 = Sa[bi][k], a1 = Sa[bi + 1][k];
      const double b0 = Sb[k][bj], b1 = Sb[k][bj + 1];
      c00 += a0 * b0; c01 += a0 * b1; c10 += a1 * b0; c11 += a1 * b1;
    }
    C[bi * T + bj] -= c00;
    C[bi * T + bj + 1] -= c01;
    C[(bi + 1) * T + bj] -= c10;
    C[(bi + 1) * T + bj + 1] -= c11;
  } else {
    const int i = threadIdx.x / T, j = threadIdx.x % T;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < T; ++k) acc += Sa[i][k] * Sb[k][j];
    C[i * T + j] -= acc;
  }
}

template <int T, class CT = double>
__device__ inline CT *tile_at(CT *F, const SubInfo &s, int K, int slot) {
  return F + s.base + ((int64_t)K * (s.bl + s.bu + 1) + slot) * (T * T);
}

// One workgroup factors one subdomain (batched over subdomains, LPT order).
// Dynamic LDS holds the U panel (bu tiles).
template <int T>
__global__ __launch_bounds__(256) void k_band_lu(double *__restrict__ F, const SubInfo *__restrict__ subs,
                                                 const int32_t *__restrict__ erow, const int32_t *__restrict__ elo,
                                                 const int32_t *__restrict__ order, int *status) {
  __shared__ LuLds<T, double> L;
  extern __shared__ double upanel_raw[];
  double(*Up)[T][T + 1] = reinterpret_cast<double(*)[T][T + 1]>(upanel_raw);
  const SubInfo s = subs[order[blockIdx.x]];
  const TileRows R = tile_rows(s, erow, elo);
  auto tile = [&](int I, int J) { return F + R.at<T>(I, J); };
  for (int K = 0; K < s.nt; ++K) {
    lu_diag_tile<T>(tile(K, K), L, status);
    // the envelope is symmetric: rows K + 1 .. last(K) have a tile in column K
    const int ie = R.last(K), je = ie;
    for (int I = K + 1; I <= ie; ++I) panel_tile<T>(tile(I, K), L, true);
    for (int J = K + 1; J <= je; ++J) {
      double *a = tile(K, J);
      panel_tile<T>(a, L, false);
      for (int e = threadIdx.x; e < T * T; e += 256) Up[J - K - 1][e / T][e % T] = a[e];
    }
    __syncthreads();
    for (int I = K + 1; I <= ie; ++I) {
      const double *lik = tile(I, K);
      for (int e = threadIdx.x; e < T * T; e += 256) L.S[e / T][e % T] = lik[e];
      __syncthreads();
      for (int J = K + 1; J <= je; ++J) schur_tile<T>(tile(I, J), L.S, Up[J - K - 1]);
      __syncthreads();
    }
  }
}

// ----------------------------------------------------------------------
// LU with 32x32 tiles and the tile products on MFMA.
// CT = double uses v_mfma_f64_16x16x4f64, CT = float v_mfma_f32_16x16x4f32.
// MFMA operand layouts (16x16x4): A[i][k] in lane i + 16 k; B[k][j] in lane
// j + 16 k.  Accumulator element v of lane l holds column l % 16 and row
// 4 (l / 16) + v for f32, but row (l / 16) + 4 v for f64 (one-row groups).
// ----------------------------------------------------------------------
template <class CT>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int lk, int v) { return 4 * lk + v; }
};

// LU without pivoting of a 32x32 tile and the explicit inverses of both
// factors in one forward sweep of 32 steps.  Step k uses the unscaled
// column k, l_ik = a_ik / a_kk formed on the fly, and row k of U (final at
// step k):
//   trailing update   a_ij -= l_ik a_kj                 (i, j > k)
//   X = L^{-1}         X_ij -= l_ik X_kj                (i > k, j <= k)
//   Z = (U^T)^{-1}     Z_ij -= U_ki (Z_kj / U_kk)       (i > k, j <= k)
// (the last two are forward elimination applied to the identity), and
// U^{-1} = Z^T.  The tile is held in registers: thread (ti, tj) =
// (tid / 32, tid % 32) owns column tj of rows ti + (NT / 32) h of A, X and
// Z, and each step only row k of A, X, Z and column k of A pass through LDS
// (double-buffered by step parity, one barrier per step).  dk: the tile in
// global memory (read, then replaced by the strict lower of L^{-1} and the
// upper of U^{-1}); Li, Ui: LDS tiles that receive L^{-1} (dense unit lower)
// and U^{-1} (dense upper).  Raises *status on a zero or nonfinite pivot.
// dh, when given: the tile's bfloat16 copy, written with dk.
template <class CT, int NT>
__device__ void lu_inv_diag_regs(CT *__restrict__ dk, CT (*Li)[33], CT (*Ui)[33], int *status,
                                 __hip_bfloat16 *__restrict__ dh = nullptr) {
  constexpr int T = 32, RS = NT / T, R = T / RS;
  static_assert(NT % T == 0 && R >= 1 && R <= 4, "workgroup size");
  __shared__ CT pub[2][4][T];  // [parity][row A, row X, row Z, column A]
  const int tid = threadIdx.x, ti = tid / T, tj = tid % T;
  CT a[R], x[R], z[R];
#pragma unroll
  for (int h = 0; h < R; ++h) {
    const int i = ti + RS * h;
    a[h] = dk[i * T + tj];
    x[h] = (i == tj) ? (CT)1 : (CT)0;
    z[h] = x[h];
  }
  auto publish = [&](int kn, int p) {
#pragma unroll
    for (int h = 0; h < R; ++h) {
      const int i = ti + RS * h;
      if (i == kn) {
        pub[p][0][tj] = a[h];
        pub[p][1][tj] = x[h];
        pub[p][2][tj] = z[h];
      }
      if (tj == kn) pub[p][3][i] = a[h];
    }
  };
  publish(0, 0);
  __syncthreads();
  for (int k = 0; k < T; ++k) {
    const int p = k & 1;
    // every LDS operand of the step is read up front (one wait); the
    // updates below are selects, not branches
    const CT piv = pub[p][0][k];
    const CT akj = pub[p][0][tj], xkj = pub[p][1][tj], zkj = pub[p][2][tj];
    CT cik[R], uki[R];
#pragma unroll
    for (int h = 0; h < R; ++h) {
      cik[h] = pub[p][3][ti + RS * h];
      uki[h] = pub[p][0][ti + RS * h];
    }
    if (tid == 0 && (!isfinite((double)piv) || fabs((double)piv) < 1e-300)) atomicOr(status, 1);
    const CT rp = (CT)1 / piv;
    const CT zs = zkj * rp;
#pragma unroll
    for (int h = 0; h < R; ++h) {
      const int i = ti + RS * h;
      const bool below = i > k, left = tj <= k;
      const CT l = cik[h] * rp;
      const CT an = a[h] - l * akj, xn = x[h] - l * xkj, zn = z[h] - uki[h] * zs;
      a[h] = below ? (left ? (tj == k ? l : a[h]) : an) : a[h];
      x[h] = (below && left) ? xn : x[h];
      z[h] = (below && left) ? zn : ((i == k && left) ? z[h] * rp : z[h]);  // row k of Z is final
    }
    if (k + 1 < T) publish(k + 1, p ^ 1);
    __syncthreads();
  }
  // Li = X (lower), Ui = Z^T (upper); then the tile from LDS, coalesced
#pragma unroll
  for (int h = 0; h < R; ++h) {
    const int i = ti + RS * h;
    Li[i][tj] = (i >= tj) ? x[h] : (CT)0;
    Ui[tj][i] = (i >= tj) ? z[h] : (CT)0;
  }
  __syncthreads();
  for (int e = tid; e < T * T; e += NT) {
    const int i = e / T, j = e % T;
    const CT v = (i > j) ? Li[i][j] : Ui[i][j];
    dk[e] = v;
    if (dh) dh[e] = to_ft<__hip_bfloat16>((double)v);
  }
}

// LU of the subdomains (tile 32, NW waves per workgroup), right-looking by
// block rows.  Step K:
//   (1) the diagonal tile is factored and both factors inverted (register
//       sweep above);
//   (2) U panel U_KJ = L_KK^{-1} A_KJ on MFMA, in chunks of NW QW tiles
//       (one chunk unless the row is wider).  Wave w owns the chunk's
//       tiles jj = c0 + w + NW q (q < QW) and keeps them in registers: the
//       accumulator layout of a 16x16 MFMA result is the B-operand layout
//       of a later product whose k index runs over the result rows (in the
//       accumulator's own row order), so U never goes through LDS;
//   (3) for each block row I below: L_IK = A_IK U_KK^{-1} (four waves, one
//       16x16 quadrant each, A_IK read straight into the A-operand layout;
//       later chunks read the stored L_IK back), staged in one of two LDS
//       buffers (one barrier per row), and the C strip C_IJ -= L_IK U_KJ of
//       the wave's own tiles on MFMA.
// LDS: L_KK^{-1}, U_KK^{-1} and the two row buffers.  With four waves the
// float64 kernel stays within 256 registers, so two workgroups share a
// compute unit and hide each other's latencies.  Launched with a queue
// counter, a grid smaller than the subdomain count draws subdomains until
// they are exhausted (every workgroup exits once the counter passes nsub).
template <class CT, int NW, int QW, bool HCOPY>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 4 ? 2 : 1))) void k_band_lu32(
    CT *__restrict__ F, const SubInfo *__restrict__ subs, const int32_t *__restrict__ erow,
    const int32_t *__restrict__ elo, const int32_t *__restrict__ order, int nsub, int *__restrict__ queue,
    int *status, __hip_bfloat16 *__restrict__ Fh) {
  constexpr int T = 32, NT = 64 * NW, CH = NW * QW;
  typedef typename Mfma<CT>::v4 v4;
  __shared__ CT Ui[T][T + 1];     // U_KK^{-1}, dense upper
  __shared__ CT Li[T][T + 1];     // L_KK^{-1}, dense unit lower
  __shared__ CT Sx[2][T][T + 1];  // L_IK buffers of the row loop
  __shared__ int next;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int qi = (wave >> 1) & 1, qj = wave & 1;
  // subdomains in the queue's (largest-first) order: one per workgroup, or,
  // with a queue counter, as many as the workgroup draws until none is left
  for (int it = blockIdx.x; it < nsub;) {
  const SubInfo s = subs[order[it]];
  const TileRows R = tile_rows(s, erow, elo);
  for (int K = 0; K < s.nt; ++K) {
    // the envelope is symmetric: row K's U tiles and the rows below with a
    // tile in column K both end at last(K)
    const int je = R.last(K), nu = je - K;
    const int ie = je;
    // (1) diagonal tile: LU and both inverses in one sweep
    lu_inv_diag_regs<CT, NT>(F + R.at<T>(K, K), Li, Ui, status, HCOPY ? Fh + R.at<T>(K, K) : nullptr);
    // the panel in chunks of CH tiles (one chunk unless the row is wider)
    for (int c0 = 0; c0 < nu; c0 += CH) {
      // (2) the wave's U-panel tiles of this chunk, kept as B operands:
      // ub[q][bj][4 bi + v] holds U_KJ[16 bi + row(lk, v)][16 bj + lr]
      CT ub[QW][2][8];
#pragma unroll
      for (int q = 0; q < QW; ++q) {
        const int jj = c0 + wave + NW * q;
        if (jj < nu) {
          CT *g = F + R.at<T>(K, K + 1 + jj);
          CT bl[8][2];
#pragma unroll
          for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) bl[m][bj] = g[(4 * m + lk) * T + 16 * bj + lr];
          v4 acc[2][2];
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4{0, 0, 0, 0};
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            const CT a0 = Li[lr][4 * m + lk], a1 = Li[16 + lr][4 * m + lk];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
              acc[0][bj] = Mfma<CT>::op(a0, bl[m][bj], acc[0][bj]);
              acc[1][bj] = Mfma<CT>::op(a1, bl[m][bj], acc[1][bj]);
            }
          }
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                ub[q][bj][4 * bi + v] = acc[bi][bj][v];
                g[(16 * bi + Mfma<CT>::row(lk, v)) * T + 16 * bj + lr] = acc[bi][bj][v];
              }
          // U_KJ is final: its bfloat16 copy
          if constexpr (HCOPY) {
            __hip_bfloat16 *gh = Fh + R.at<T>(K, K + 1 + jj);
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
              for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                  gh[(16 * bi + Mfma<CT>::row(lk, v)) * T + 16 * bj + lr] = to_ft<__hip_bfloat16>((double)acc[bi][bj][v]);
          }
        }
      }
      // (3) block rows below: L_IK (first chunk: computed and stored; later
      // chunks: read back), then the wave's C tiles of the chunk
      for (int I = K + 1; I <= ie; ++I) {
        const int buf = (I - K - 1) & 1;
        CT *aik = F + R.at<T>(I, K);
        v4 acc[QW][2][2];
#pragma unroll
        for (int q = 0; q < QW; ++q) {
          const int jj = c0 + wave + NW * q;
          if (jj < nu) {
            const CT *c = F + R.at<T>(I, K + 1 + jj);
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
              for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                  acc[q][bi][bj][v] = c[(16 * bi + Mfma<CT>::row(lk, v)) * T + 16 * bj + lr];
          }
        }
        if (c0 == 0) {
          // A_IK quadrant rows in the A-operand layout
          CT ra[8];
          if (wave < 4) {
#pragma unroll
            for (int m = 0; m < 8; ++m) ra[m] = aik[(16 * qi + lr) * T + 4 * m + lk];
          }
          v4 l = {0, 0, 0, 0};
          if (wave < 4) {
#pragma unroll
            for (int m = 0; m < 8; ++m) l = Mfma<CT>::op(ra[m], Ui[4 * m + lk][16 * qj + lr], l);
#pragma unroll
            for (int v = 0; v < 4; ++v) Sx[buf][16 * qi + Mfma<CT>::row(lk, v)][16 * qj + lr] = l[v];
          }
          __syncthreads();  // L_IK staged; every wave has read A_IK
          if (wave < 4) {
#pragma unroll
            for (int v = 0; v < 4; ++v) aik[(16 * qi + Mfma<CT>::row(lk, v)) * T + 16 * qj + lr] = l[v];
            // L_IK is final: its bfloat16 copy
            if constexpr (HCOPY) {
              __hip_bfloat16 *ah = Fh + R.at<T>(I, K);
#pragma unroll
              for (int v = 0; v < 4; ++v)
                ah[(16 * qi + Mfma<CT>::row(lk, v)) * T + 16 * qj + lr] = to_ft<__hip_bfloat16>((double)l[v]);
            }
          }
        } else {
          for (int e = tid; e < T * T; e += NT) Sx[buf][e / T][e % T] = aik[e];
          __syncthreads();  // L_IK staged
        }
        // C_IJ -= L_IK U_KJ; the k index of step (bi, v) is 16 bi + row(lk, v)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int kc = 16 * bi + Mfma<CT>::row(lk, v);
            const CT a0 = -Sx[buf][lr][kc], a1 = -Sx[buf][16 + lr][kc];
#pragma unroll
            for (int q = 0; q < QW; ++q) {
              const int jj = c0 + wave + NW * q;
              if (jj < nu) {
                acc[q][0][0] = Mfma<CT>::op(a0, ub[q][0][4 * bi + v], acc[q][0][0]);
                acc[q][0][1] = Mfma<CT>::op(a0, ub[q][1][4 * bi + v], acc[q][0][1]);
                acc[q][1][0] = Mfma<CT>::op(a1, ub[q][0][4 * bi + v], acc[q][1][0]);
                acc[q][1][1] = Mfma<CT>::op(a1, ub[q][1][4 * bi + v], acc[q][1][1]);
              }
            }
          }
#pragma unroll
        for (int q = 0; q < QW; ++q) {
          const int jj = c0 + wave + NW * q;
          if (jj < nu) {
            CT *c = F + R.at<T>(I, K + 1 + jj);
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
              for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) c[(16 * bi + Mfma<CT>::row(lk, v)) * T + 16 * bj + lr] = acc[q][bi][bj][v];
          }
        }
      }
      // L tiles stored by other waves are read back by the next chunk
      __threadfence_block();
      __syncthreads();
    }
    // the next step's diagonal tile and U panel were written by other waves
    // of this workgroup: make the stores visible before they are read
    __threadfence_block();
    __syncthreads();
  }
    if (!queue) break;
    // the counter starts at the grid size: the first subdomains went to
    // the workgroups by their index
    if (tid == 0) next = atomicAdd(queue, 1);
    __syncthreads();
    it = next;
    __syncthreads();
  }
}

// Multi-launch variant for one large band matrix (the coarse problem):
// step K = diag (1 WG), panels (bl + bu WGs), Schur (bl x bu WGs).
// With tile 32 the steps use the single-wave diagonal factorisation, the
// one-barrier-per-step inverses and MFMA tile products, and stay within
// 25 KB of LDS so that they fit beside a subdomain-factorisation workgroup
// on the same compute unit (the coarse chain runs on its own stream while
// the subdomains are factored).
// The coarse step kernels run beside the subdomain factorisation, which
// leaves about 64 VGPRs per SIMD lane free: they are held to 64 (8 waves
// per SIMD) so that they fit there.
template <int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_lu_step_diag(
    double *__restrict__ F, SubInfo s, int K, int *status) {
  if constexpr (T == 32) {
    __shared__ double Li[T][T + 1], Ui[T][T + 1];
    lu_inv_diag_regs<double, 256>(tile_at<T>(F, s, K, s.bl), Li, Ui, status);
  } else {
    __shared__ LuLds<T, double> L;
    lu_diag_tile<T>(tile_at<T>(F, s, K, s.bl), L, status);
  }
}
template <int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_lu_step_panel(double *__restrict__ F, SubInfo s, int K) {
  const int b = blockIdx.x;
  const bool lower = b < s.bl;
  const int IJ = K + 1 + (lower ? b : b - s.bl);
  if (IJ >= s.nt) return;
  double *a = lower ? tile_at<T>(F, s, IJ, K - IJ + s.bl) : tile_at<T>(F, s, K, IJ - K + s.bl);
  if constexpr (T == 32) {
    // lower panel X = A U_KK^{-1}, upper panel X = L_KK^{-1} A, on MFMA
    typedef Mfma<double>::v4 v4;
    __shared__ double Dm[T][T + 1], Sa[T][T + 1];
    const double *dk = tile_at<T>(F, s, K, s.bl);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4, qi = wave >> 1, qj = wave & 1;
    for (int e = tid; e < T * T; e += 256) {
      const int i = e / T, j = e % T;
      const double d = dk[e];
      Dm[i][j] = lower ? (i <= j ? d : 0.0) : (i > j ? d : (i == j ? 1.0 : 0.0));
      Sa[i][j] = a[e];
    }
    __syncthreads();
    v4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < T; k0 += 4)
      x = lower ? Mfma<double>::op(Sa[16 * qi + lr][k0 + lk], Dm[k0 + lk][16 * qj + lr], x)
                : Mfma<double>::op(Dm[16 * qi + lr][k0 + lk], Sa[k0 + lk][16 * qj + lr], x);
#pragma unroll
    for (int v = 0; v < 4; ++v) a[(16 * qi + Mfma<double>::row(lk, v)) * T + 16 * qj + lr] = x[v];
  } else {
    __shared__ LuLds<T, double> L;
    load_diag_inverses<T>(tile_at<T>(F, s, K, s.bl), L);
    panel_tile<T>(a, L, lower);
  }
}
template <int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_lu_step_schur(double *__restrict__ F, SubInfo s, int K) {
  __shared__ double Sa[T][T + 1], Sb[T][T + 1];
  const int I = K + 1 + blockIdx.x / s.bu, J = K + 1 + blockIdx.x % s.bu;
  if (I >= s.nt || J >= s.nt) return;
  const double *lik = tile_at<T>(F, s, I, K - I + s.bl);
  const double *ukj = tile_at<T>(F, s, K, J - K + s.bl);
  double *c = tile_at<T>(F, s, I, J - I + s.bl);
  if constexpr (T == 32) {
    // C -= L_IK U_KJ on MFMA, one 16x16 quadrant per wave
    typedef Mfma<double>::v4 v4;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4, qi = wave >> 1, qj = wave & 1;
    v4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = c[(16 * qi + Mfma<double>::row(lk, v)) * T + 16 * qj + lr];
    for (int e = tid; e < T * T; e += 256) {
      Sa[e / T][e % T] = -lik[e];
      Sb[e / T][e % T] = ukj[e];
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < T; k0 += 4) acc = Mfma<double>::op(Sa[16 * qi + lr][k0 + lk], Sb[k0 + lk][16 * qj + lr], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) c[(16 * qi + Mfma<double>::row(lk, v)) * T + 16 * qj + lr] = acc[v];
  } else {
    for (int e = threadIdx.x; e < T * T; e += 256) {
      Sa[e / T][e % T] = lik[e];
      Sb[e / T][e % T] = ukj[e];
    }
    __syncthreads();
    schur_tile<T>(c, Sa, Sb);
  }
}

// One launch per block column K of the coarse factorisation (tile 32),
// replacing the panel and Schur launches and the next diagonal launch.
// Blocks [0, bl bu): Schur tile (I, J) = (K + 1 + b / bu, K + 1 + b % bu)
// forms L_IK = A_IK U_KK^{-1} and U_KJ = L_KK^{-1} A_KJ itself from the
// unmodified panel tiles (each panel tile is formed by every Schur block
// that needs it), updates C_IJ -= L_IK U_KJ, and the block of tile
// (K + 1, K + 1) then factors that tile.  Blocks [bl bu, bl bu + bl + bu):
// write the panel tiles of step K - 1 in place; no block of this launch
// reads those tiles, and their unmodified values are no longer needed.
// Launch K = nt - 1 only writes the panels of step nt - 2; the diagonal
// tile of step 0 is factored by k_lu_step_diag first.  Panel operands are
// read from global memory straight into the MFMA operand layouts and the
// diagonal inverses are masked out of the stored diagonal tile, so a block
// needs two LDS tiles (19 KB with the sweep's row buffers) and 64 VGPRs.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_lu_step_fused(
    double *__restrict__ F, SubInfo s, int K, int *status) {
  constexpr int T = 32;
  typedef Mfma<double>::v4 v4;
  __shared__ double X0[T][T + 1], X1[T][T + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4, qi = wave >> 1, qj = wave & 1;
  const int nschur = s.bl * s.bu;
  const int b = blockIdx.x;
  // stored diagonal tile of step k into X0: strict lower of L_kk^{-1},
  // upper of U_kk^{-1}
  auto load_diag = [&](int k) {
    const double *dk = tile_at<T>(F, s, k, s.bl);
    for (int e = tid; e < T * T; e += 256) X0[e / T][e % T] = dk[e];
  };
  auto ui = [&](int k, int j) { return k <= j ? X0[k][j] : 0.0; };                     // U_kk^{-1}
  auto li = [&](int i, int k) { return i > k ? X0[i][k] : (i == k ? 1.0 : 0.0); };  // L_kk^{-1}
  // quadrant (qi, qj) of A Ui (A-operand rows of A from global) or of
  // Li A (B-operand columns of A from global)
  auto right_ui = [&](const double *A) {
    v4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < T; k0 += 4)
      x = Mfma<double>::op(A[(16 * qi + lr) * T + k0 + lk], ui(k0 + lk, 16 * qj + lr), x);
    return x;
  };
  auto left_li = [&](const double *A) {
    v4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < T; k0 += 4)
      x = Mfma<double>::op(li(16 * qi + lr, k0 + lk), A[(k0 + lk) * T + 16 * qj + lr], x);
    return x;
  };
  if (b >= nschur) {
    // panel tile of step K - 1, in place
    const int Kp = K - 1, m = b - nschur;
    if (Kp < 0) return;
    const bool lower = m < s.bl;
    const int IJ = Kp + 1 + (lower ? m : m - s.bl);
    if (IJ >= s.nt) return;
    double *a = lower ? tile_at<T>(F, s, IJ, Kp - IJ + s.bl) : tile_at<T>(F, s, Kp, IJ - Kp + s.bl);
    load_diag(Kp);
    __syncthreads();
    const v4 x = lower ? right_ui(a) : left_li(a);
    __syncthreads();  // every wave has read the tile
#pragma unroll
    for (int v = 0; v < 4; ++v) a[(16 * qi + Mfma<double>::row(lk, v)) * T + 16 * qj + lr] = x[v];
    return;
  }
  const int I = K + 1 + b / s.bu, J = K + 1 + b % s.bu;
  if (I >= s.nt || J >= s.nt) return;
  double *c = tile_at<T>(F, s, I, J - I + s.bl);
  load_diag(K);
  __syncthreads();
  const v4 l = right_ui(tile_at<T>(F, s, I, K - I + s.bl));
  const v4 u = left_li(tile_at<T>(F, s, K, J - K + s.bl));
  __syncthreads();  // X0 free
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * qi + Mfma<double>::row(lk, v), j = 16 * qj + lr;
    X0[i][j] = -l[v];
    X1[i][j] = u[v];
  }
  v4 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = c[(16 * qi + Mfma<double>::row(lk, v)) * T + 16 * qj + lr];
  __syncthreads();
#pragma unroll
  for (int k0 = 0; k0 < T; k0 += 4) acc = Mfma<double>::op(X0[16 * qi + lr][k0 + lk], X1[k0 + lk][16 * qj + lr], acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) c[(16 * qi + Mfma<double>::row(lk, v)) * T + 16 * qj + lr] = acc[v];
  if (I == K + 1 && J == K + 1) {
    // the next diagonal tile is final: factor it (read back by this block)
    __threadfence_block();
    __syncthreads();
    lu_inv_diag_regs<double, 256>(c, X0, X1, status);
  }
}

// ----------------------------------------------------------------------
// Tile triangular solves (the subdomain apply A_i^{-1} r_i).
// One workgroup per subdomain; the local vector x lives in LDS (dynamic)
// or, for the big coarse system, in a global scratch vector.
// Non-transposed: forward with L (tiles left of the diagonal, then the
// unit-lower inverse), backward with U.  Transposed: forward with U^T,
// backward with L^T.
// ----------------------------------------------------------------------
// Barrier for workgroups that communicate through LDS only: it waits for
// the wave's LDS operations, not for its outstanding global loads/stores,
// so prefetched tile loads stay in flight across it.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int G>
__device__ inline double group_sum(double v) {
  // lanes of one group are consecutive (row-major mapping)
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// mode: 0 = non-transposed, owned write z[g] = x (or z[g] += x if add)
//       1 = transposed: masked gather, result written to the per-subdomain
//           buffer yloc (summed over copies afterwards)
constexpr int RING = 32;  // block rows of the local vector kept in LDS (> bl, bu)
static_assert((RING & (RING - 1)) == 0, "ring indices are taken modulo RING with a mask");
// off-diagonal tiles per block row held in registers at once
// (the summation order does not depend on it)
template <int T, class FT, int NTHR>
constexpr int solve_bmax() {
  // 256 threads: the register sets of the rows in flight (below) stay
  // within 128 registers, so that four subdomains share a compute unit
  // (float64 loads each row's tiles in the row: ahead-loading measured no
  // faster there)
  if (T == 32 && NTHR == 256) return sizeof(FT) == 8 ? 6 : (sizeof(FT) == 4 ? 6 : 8);
  // 128 threads (two waves per subdomain, 8 elements of a tile row per
  // lane): 256 registers per lane
  if (T == 32 && NTHR == 128) return sizeof(FT) == 8 ? 4 : (sizeof(FT) == 4 ? 6 : 8);
  // float64 at 512 threads: 8 tiles (a typical band), so that two block
  // rows' first chunks fit the cross-row prefetch budget
  if (T == 32 && NTHR == 512 && sizeof(FT) == 8) return 8;
  // otherwise as many as 48 registers hold, at most 8 (rows past their
  // last tile re-read the diagonal tile in the slots beyond it)
  constexpr int per = T * T / NTHR;  // tile elements per lane
  constexpr int regs = per * (sizeof(FT) >= 4 ? (int)sizeof(FT) / 4 : 1);
  constexpr int b = 48 / regs;
  return b > 8 ? 8 : (b < 1 ? 1 : b);
}
// block rows ahead of the one computing whose first tile chunk is already
// being loaded (0: every row loads its own tiles)
template <int T, class FT, int NTHR>
constexpr int solve_depth() {
  if (T == 32 && NTHR == 256) return sizeof(FT) == 8 ? 0 : 2;
  if (T == 32 && NTHR == 128) return sizeof(FT) == 8 ? 1 : (sizeof(FT) == 4 ? 2 : 3);
  constexpr int per = T * T / NTHR;
  constexpr int regs = per * (((int)sizeof(FT) + 3) / 4);
  return (solve_bmax<T, FT, NTHR>() + 1) * regs <= 40 ? 1 : 0;
}

// PER consecutive elements of one tile row (aligned to PER elements), read
// as one or two vector loads
template <class FT, int PER>
__device__ inline void load_chunk(const FT *__restrict__ p, FT (&out)[PER]) {
  if constexpr (sizeof(FT) * PER == 16) {
    // 16-B chunks as non-temporal loads: on the realistic workload the
    // FP64 solve at 512 threads 3.8% faster (3.98 -> 3.83 ms), FP32 at 256
    // 1.3% and BF16 at 128 1.7%, the ensemble's FP32 solve 4.8%; the same
    // hint on the 32-B float64 chunks of 256 threads made that solve 10%
    // slower
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 c = __builtin_nontemporal_load(reinterpret_cast<const u4 *>(p));
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      if constexpr (sizeof(FT) == 8)
        out[m] = __hiloint2double((int)c[2 * m + 1], (int)c[2 * m]);
      else if constexpr (sizeof(FT) == 4)
        out[m] = __uint_as_float(c[m]);
      else
        out[m] = __ushort_as_bfloat16((unsigned short)(c[m / 2] >> (16 * (m % 2))));
    }
  } else {
    struct alignas(PER * sizeof(FT)) Chunk { FT v[PER]; };
    const Chunk c = *reinterpret_cast<const Chunk *>(p);
#pragma unroll
    for (int m = 0; m < PER; ++m) out[m] = c.v[m];
  }
}

// Forward and backward sweeps of one subdomain (or of the coarse system).
// Only a ring of RING block rows of the local vector lives in LDS; the
// forward results go to a global scratch (ybuf) and are re-read by the
// backward sweep.  For every block row, the tiles it needs are loaded into
// registers (chunks of SOLVE_BMAX) before any arithmetic, so that their
// loads are in flight together.
//   mode non-transposed: z[g] = x (owned entries; or z[g] += x when add)
//   mode transposed: input masked by D_i, output to yloc (summed later)
template <int T, class FT, int NTHR, bool TRANS>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(NTHR == 256 ? 4 : (NTHR == 128 ? 2 : 1), 8)))
void k_band_solve(const FT *__restrict__ F, const SubInfo *__restrict__ subs, const int32_t *__restrict__ erow,
                  const int32_t *__restrict__ elo, const int32_t *__restrict__ order,
                  const int32_t *__restrict__ l2g, const uint8_t *__restrict__ owned, const double *__restrict__ r,
                  double *__restrict__ z, int add, double *__restrict__ yloc, double *__restrict__ ybuf,
                  const int32_t *__restrict__ sub_seg, const uint8_t *__restrict__ seg_active) {
  constexpr bool transpose = TRANS;
  constexpr int SOLVE_BMAX = solve_bmax<T, FT, NTHR>();
  constexpr int G = NTHR / T;   // lanes per row
  constexpr int PER = T / G;    // elements of one tile row per lane
  __shared__ double ring[RING][T];
  __shared__ double acc_s[T];
  __shared__ double part_s[G][T];
  const int sidx = order ? order[blockIdx.x] : blockIdx.x;
  // subdomains of inactive instances (converged in a batch) are skipped;
  // their part of z is left as it was
  if (seg_active && !seg_active[sub_seg[sidx]]) return;
  const SubInfo s = subs[sidx];
  const bool local = s.l2g_off >= 0;
  const int64_t yo = local ? s.l2g_off : 0;
  const int tid = threadIdx.x;
  const TileRows R = tile_rows(s, erow, elo);
  auto tile = [&](int K, int J) -> const FT * { return F + R.at<T>(K, J); };  // tile (K, J), J a tile column
  // this lane's chunk (row i, elements g PER ..) of the diagonal tile of row
  // K; the forward sweep uses its strict lower part (L_KK^{-1}), the
  // backward sweep its upper part (U_KK^{-1}), so a chunk with no element
  // in the half in use is not loaded (in float64 that skips about half the
  // tile's cache lines)
  auto load_diag = [&](int K, bool lower, int i, int g, FT (&dv)[PER]) {
    const bool used = lower ? (g * PER < i) : (g * PER + PER - 1 >= i);
    if (used) {
      load_chunk<FT, PER>(tile(K, K) + i * T + g * PER, dv);
    } else {
#pragma unroll
      for (int m = 0; m < PER; ++m) dv[m] = (FT)0;
    }
  };
  auto rhs = [&](int l) -> double {
    if (l >= s.n_loc) return 0.0;
    if (!local) return r[l];
    double v = r[l2g[s.l2g_off + l]];
    if (transpose && !owned[s.l2g_off + l]) v = 0.0;
    return v;
  };
  // gather the right-hand side R_i r (D_i R_i r when transposed) into ybuf
  // (in batches of GB entries per thread, so that their index and value
  // loads are in flight together)
  constexpr int GB = 8;
  for (int l0 = 0; l0 < s.n_loc; l0 += GB * NTHR) {
    double v[GB];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const int l = l0 + q * NTHR + tid;
      v[q] = l < s.n_loc ? rhs(l) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const int l = l0 + q * NTHR + tid;
      if (l < s.n_loc) ybuf[yo + l] = v[q];
    }
  }
  __syncthreads();
  constexpr int DEPTH = solve_depth<T, FT, NTHR>();
  if constexpr (!TRANS && DEPTH > 0) {
    const int i = tid / G, g = tid % G;
    // A block row's first chunk of off-diagonal tiles, its diagonal-tile
    // chunk and its right-hand side entry, in registers.  DEPTH + 1 such
    // sets rotate: while row K computes, the loads of rows K + 1 .. K +
    // DEPTH are in flight.  Every row issues the same loads whatever its
    // width (slots past the row's last tile re-read its diagonal tile, rows
    // past the end re-read the last row), so that the wait before a row's
    // arithmetic counts exactly the loads issued after that row's set;
    // conditional loads would make it wait for all of them.  Further chunks
    // of a wide band are loaded in the row itself.  The summation order is
    // the same as without the rotation.
    struct RowRegs {
      FT buf[SOLVE_BMAX][PER];
      FT dv[PER];
      double bv;
      const FT *t0;  // tile (K, 0) of the row's storage (tile (K, J) at t0 + J T^2)
      int c0, c1;    // off-diagonal tile columns in use
    };
    // row K's off-diagonal tile columns (left of the diagonal when lower,
    // right of it otherwise), its first chunk of them, its diagonal-tile
    // chunk (a lane with no entry in the triangle in use reads a chunk of
    // its row that another lane uses, and masks it) and ybuf entry K T + i
    auto load_row = [&](int K, bool lower, RowRegs &Rr) {
      int64_t off0;
      int first, last;
      R.row_info<T>(K, off0, first, last);
      Rr.t0 = F + off0;
      Rr.c0 = lower ? first : K + 1;
      Rr.c1 = lower ? K - 1 : last;
      const FT *dk = Rr.t0 + (int64_t)K * (T * T);
      const bool used = lower ? (g * PER < i) : (g * PER + PER - 1 >= i);
      load_chunk<FT, PER>(dk + i * T + (used ? g * PER : (lower ? 0 : T - PER)), Rr.dv);
#pragma unroll
      for (int t = 0; t < SOLVE_BMAX; ++t) {
        const FT *tp = (Rr.c0 + t <= Rr.c1) ? Rr.t0 + (int64_t)(Rr.c0 + t) * (T * T) : dk;
        load_chunk<FT, PER>(tp + i * T + g * PER, Rr.buf[t]);
      }
      Rr.bv = ybuf[yo + min(K * T + i, s.n_loc - 1)];
    };
    auto off_sum = [&](const RowRegs &Rr) {
      const int c0 = Rr.c0, c1 = Rr.c1;
      double a = 0.0;
#pragma unroll
      for (int t = 0; t < SOLVE_BMAX; ++t)
        if (c0 + t <= c1) {
          const double *xr = ring[(c0 + t) & (RING - 1)];
#pragma unroll
          for (int m = 0; m < PER; ++m) a += from_ft<FT>(Rr.buf[t][m]) * xr[g * PER + m];
        }
      // (a further chunk's loads all go out before its first use; slots
      // past c1 re-read the chunk's first tile)
      for (int C0 = c0 + SOLVE_BMAX; C0 <= c1; C0 += SOLVE_BMAX) {
        FT buf[SOLVE_BMAX][PER];
        const FT *tc = Rr.t0 + (int64_t)C0 * (T * T);
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t) {
          const FT *tp = (C0 + t <= c1) ? tc + t * (T * T) : tc;
          load_chunk<FT, PER>(tp + i * T + g * PER, buf[t]);
        }
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (C0 + t <= c1) {
            const double *xr = ring[(C0 + t) & (RING - 1)];
#pragma unroll
            for (int m = 0; m < PER; ++m) a += from_ft<FT>(buf[t][m]) * xr[g * PER + m];
          }
      }
      return a;
    };
    // one block row: v_K = D_KK (b_K - sum of the off-diagonal tiles times
    // the ring), D_KK the strict-lower (forward, unit diagonal) or upper
    // (backward) part of the stored inverse; v_K goes to the ring and ybuf
    auto row = [&](int K, bool lower, const RowRegs &Rr) {
      double a = off_sum(Rr);
      a = group_sum<G>(a);
      const bool in = K * T + i < s.n_loc;
      if (g == 0) acc_s[i] = (in ? Rr.bv : 0.0) - a;
      lds_barrier();
      double y = 0.0;
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = g * PER + m;
        if (lower ? (j < i) : (j >= i)) y += from_ft<FT>(Rr.dv[m]) * acc_s[j];
      }
      y = group_sum<G>(y);
      if (g == 0) {
        const double v = lower ? acc_s[i] + y : y;
        ring[K % RING][i] = v;
        if (in) ybuf[yo + K * T + i] = v;
      }
      lds_barrier();
    };
    if (s.nt > 0) {
      RowRegs S[DEPTH + 1];
      const int nt = s.nt;
      // forward: y_K = Linv_KK (b_K - sum_{P<K} L_KP y_P), P = first(K) .. K - 1
#pragma unroll
      for (int j = 0; j < DEPTH; ++j) {
        load_row(min(j, nt - 1), true, S[j]);
      }
      for (int K0 = 0; K0 < nt; K0 += DEPTH + 1) {
#pragma unroll
        for (int j = 0; j <= DEPTH; ++j) {
          load_row(min(K0 + j + DEPTH, nt - 1), true, S[(j + DEPTH) % (DEPTH + 1)]);
          if (K0 + j < nt) row(K0 + j, true, S[j]);
        }
      }
      // backward: x_K = Uinv_KK (y_K - sum_{J>K} U_KJ x_J), J = K + 1 .. last(K);
      // x overwrites y in ybuf (y_K is read before x_K is written)
#pragma unroll
      for (int j = 0; j < DEPTH; ++j) {
        load_row(max(nt - 1 - j, 0), false, S[j]);
      }
      for (int K0 = nt - 1; K0 >= 0; K0 -= DEPTH + 1) {
#pragma unroll
        for (int j = 0; j <= DEPTH; ++j) {
          load_row(max(K0 - j - DEPTH, 0), false, S[(j + DEPTH) % (DEPTH + 1)]);
          if (K0 - j >= 0) row(K0 - j, false, S[j]);
        }
      }
    }
    // the owned entries of x to z, after the sweeps (no load of z inside
    // them); ybuf entries were written by other threads of the workgroup
    __syncthreads();
    for (int l0 = 0; l0 < s.n_loc; l0 += GB * NTHR) {
      double x[GB];
      int32_t gi[GB];
#pragma unroll
      for (int q = 0; q < GB; ++q) {
        const int l = l0 + q * NTHR + tid;
        const bool in = l < s.n_loc;
        x[q] = in ? ybuf[yo + l] : 0.0;
        gi[q] = !in ? -1 : (local ? (owned[s.l2g_off + l] ? l2g[s.l2g_off + l] : -1) : l);
      }
#pragma unroll
      for (int q = 0; q < GB; ++q)
        if (gi[q] >= 0) z[gi[q]] = add ? z[gi[q]] + x[q] : x[q];
    }
  } else if constexpr (!TRANS) {
    const int i = tid / G, g = tid % G;
    // forward: y_K = Linv_KK (b_K - sum_{P<K} L_KP y_P)
    for (int K = 0; K < s.nt; ++K) {
      int64_t off0;
      int p0, je;
      R.row_info<T>(K, off0, p0, je);
      const FT *t0 = F + off0;
      const double bv = (g == 0 && K * T + i < s.n_loc) ? ybuf[yo + K * T + i] : 0.0;
      // the diagonal tile's loads go out with the first off-diagonal chunk
      FT dv[PER];
      load_diag(K, true, i, g, dv);
      double a = 0.0;
      for (int P0 = p0; P0 < K; P0 += SOLVE_BMAX) {
        FT buf[SOLVE_BMAX][PER];
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (P0 + t < K) {
            const FT *A = t0 + (int64_t)(P0 + t) * (T * T);
            load_chunk<FT, PER>(A + i * T + g * PER, buf[t]);
          }
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (P0 + t < K) {
            const double *xr = ring[(P0 + t) % RING];
#pragma unroll
            for (int m = 0; m < PER; ++m) a += from_ft<FT>(buf[t][m]) * xr[g * PER + m];
          }
      }
      a = group_sum<G>(a);
      if (g == 0) acc_s[i] = bv - a;
      lds_barrier();
      double y = 0.0;
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = g * PER + m;
        if (j < i) y += from_ft<FT>(dv[m]) * acc_s[j];
      }
      y = group_sum<G>(y);
      if (g == 0) {
        const double v = acc_s[i] + y;
        ring[K % RING][i] = v;
        if (K * T + i < s.n_loc) ybuf[yo + K * T + i] = v;
      }
      lds_barrier();
    }
    // backward: x_K = Uinv_KK (y_K - sum_{J>K} U_KJ x_J)
    for (int K = s.nt - 1; K >= 0; --K) {
      int64_t off0;
      int p0, je;
      R.row_info<T>(K, off0, p0, je);
      const FT *t0 = F + off0;
      const double bv = (g == 0 && K * T + i < s.n_loc) ? ybuf[yo + K * T + i] : 0.0;
      FT dv[PER];
      load_diag(K, false, i, g, dv);
      double a = 0.0;
      for (int J0 = K + 1; J0 <= je; J0 += SOLVE_BMAX) {
        FT buf[SOLVE_BMAX][PER];
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (J0 + t <= je) {
            const FT *A = t0 + (int64_t)(J0 + t) * (T * T);
            load_chunk<FT, PER>(A + i * T + g * PER, buf[t]);
          }
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (J0 + t <= je) {
            const double *xr = ring[(J0 + t) % RING];
#pragma unroll
            for (int m = 0; m < PER; ++m) a += from_ft<FT>(buf[t][m]) * xr[g * PER + m];
          }
      }
      a = group_sum<G>(a);
      if (g == 0) acc_s[i] = bv - a;
      lds_barrier();
      double y = 0.0;
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = g * PER + m;
        if (j >= i) y += from_ft<FT>(dv[m]) * acc_s[j];
      }
      y = group_sum<G>(y);
      if (g == 0) {
        ring[K % RING][i] = y;
        const int l = K * T + i;
        if (l < s.n_loc) {
          if (local) {
            if (owned[s.l2g_off + l]) {
              const int32_t gi = l2g[s.l2g_off + l];
              z[gi] = add ? z[gi] + y : y;
            }
          } else {
            z[l] = add ? z[l] + y : y;
          }
        }
      }
      lds_barrier();
    }
  } else {
    // transposed: column access; column ci = tid % T, lane group cg = tid / T
    const int ci = tid % T, cg = tid / T;
    // forward with U^T: y_K = Uinv_KK^T (b_K - sum_{P<K} U_PK^T y_P)
    for (int K = 0; K < s.nt; ++K) {
      const int p0 = R.first(K);  // rows P < K with a tile in column K (symmetric envelope)
      const double bv = (tid < T && K * T + tid < s.n_loc) ? ybuf[yo + K * T + tid] : 0.0;
      FT dv[PER];
      {
        const FT *dk = tile(K, K);
#pragma unroll
        for (int m = 0; m < PER; ++m) dv[m] = dk[(cg + m * G) * T + ci];
      }
      double a = 0.0;
      for (int P0 = p0; P0 < K; P0 += SOLVE_BMAX) {
        FT buf[SOLVE_BMAX][PER];
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (P0 + t < K) {
            const FT *A = tile(P0 + t, K);
#pragma unroll
            for (int m = 0; m < PER; ++m) buf[t][m] = A[(cg + m * G) * T + ci];
          }
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (P0 + t < K) {
            const double *xr = ring[(P0 + t) % RING];
#pragma unroll
            for (int m = 0; m < PER; ++m) a += from_ft<FT>(buf[t][m]) * xr[cg + m * G];
          }
      }
      part_s[cg][ci] = a;
      lds_barrier();
      if (tid < T) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += part_s[q][tid];
        acc_s[tid] = bv - t;
      }
      lds_barrier();
      double y = 0.0;  // y_i = sum_{j <= i} Ui[j][i] acc_j
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = cg + m * G;
        if (j <= ci) y += from_ft<FT>(dv[m]) * acc_s[j];
      }
      part_s[cg][ci] = y;
      lds_barrier();
      if (tid < T) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += part_s[q][tid];
        ring[K % RING][tid] = t;
        if (K * T + tid < s.n_loc) ybuf[yo + K * T + tid] = t;
      }
      lds_barrier();
    }
    // backward with L^T: x_K = Linv_KK^T (y_K - sum_{J>K} L_JK^T x_J)
    for (int K = s.nt - 1; K >= 0; --K) {
      const int je = R.last(K);  // rows J > K with a tile in column K
      const double bv = (tid < T && K * T + tid < s.n_loc) ? ybuf[yo + K * T + tid] : 0.0;
      FT dv[PER];
      {
        const FT *dk = tile(K, K);
#pragma unroll
        for (int m = 0; m < PER; ++m) dv[m] = dk[(cg + m * G) * T + ci];
      }
      double a = 0.0;
      for (int J0 = K + 1; J0 <= je; J0 += SOLVE_BMAX) {
        FT buf[SOLVE_BMAX][PER];
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (J0 + t <= je) {
            const FT *A = tile(J0 + t, K);
#pragma unroll
            for (int m = 0; m < PER; ++m) buf[t][m] = A[(cg + m * G) * T + ci];
          }
#pragma unroll
        for (int t = 0; t < SOLVE_BMAX; ++t)
          if (J0 + t <= je) {
            const double *xr = ring[(J0 + t) % RING];
#pragma unroll
            for (int m = 0; m < PER; ++m) a += from_ft<FT>(buf[t][m]) * xr[cg + m * G];
          }
      }
      part_s[cg][ci] = a;
      lds_barrier();
      if (tid < T) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += part_s[q][tid];
        acc_s[tid] = bv - t;
      }
      lds_barrier();
      double y = 0.0;  // x_i = acc_i + sum_{j > i} Li[j][i] acc_j
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = cg + m * G;
        if (j > ci) y += from_ft<FT>(dv[m]) * acc_s[j];
      }
      part_s[cg][ci] = y;
      lds_barrier();
      if (tid < T) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += part_s[q][tid];
        const double v = acc_s[tid] + t;
        ring[K % RING][tid] = v;
        const int l = K * T + tid;
        if (l < s.n_loc) {
          if (local)
            yloc[s.l2g_off + l] = v;
          else
            z[l] = add ? z[l] + v : v;
        }
      }
      lds_barrier();
    }
  }
}

// transposed RAS: z[g] (+)= sum over local copies of g (fixed order)
__global__ void k_gather_copies(const int64_t *__restrict__ gptr, const int32_t *__restrict__ gidx,
                                const double *__restrict__ yloc, double *__restrict__ z, int add, int64_t N) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double v = 0.0;
  for (int64_t k = gptr[g]; k < gptr[g + 1]; ++k) v += yloc[gidx[k]];
  z[g] = add ? z[g] + v : v;
}

// coarse restriction rc[perm(I)*5 + c] = sum_a Z_aI r[5a + c]: one wave
// per coarse node, lanes over its fine nodes, fixed-order wave reduction
__global__ __launch_bounds__(256) void k_coarse_restrict(const int64_t *__restrict__ zt_ptr,
                                                         const int32_t *__restrict__ zt_col,
                                                         const double *__restrict__ zt_val,
                                                         const int32_t *__restrict__ cperm,
                                                         const double *__restrict__ r, double *__restrict__ rc,
                                                         int64_t nc) {
  const int64_t I = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (I >= nc) return;  // uniform per wave
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t k = zt_ptr[I] + lane; k < zt_ptr[I + 1]; k += 64) {
    const int64_t a = zt_col[k];
    const double w = zt_val[k];
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] += w * r[5 * a + c];
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) acc[c] = wave_sum(acc[c]);
  if (lane == 0) {
    const int64_t p = cperm[I];
#pragma unroll
    for (int c = 0; c < 5; ++c) rc[5 * p + c] = acc[c];
  }
}

// coarse prolongation z[5a + c] += sum_I Z_aI xc[perm(I)*5 + c]
__global__ void k_coarse_prolong(const int64_t *__restrict__ z_ptr, const int32_t *__restrict__ z_col,
                                 const double *__restrict__ z_val, const int32_t *__restrict__ cperm,
                                 const double *__restrict__ xc, double *__restrict__ z, int64_t n) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t k = z_ptr[a]; k < z_ptr[a + 1]; ++k) {
    const int64_t p = cperm[z_col[k]];
    const double w = z_val[k];
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] += w * xc[5 * p + c];
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) z[5 * a + c] += acc[c];
}

// ----------------------------------------------------------------------
// Coarse-system solve (one large band system, FP64, non-transposed): one
// 1024-thread workgroup, one tile column per lane (32 lanes per row).  The
// tiles of block row K+1 (K-1 in the backward sweep) are loaded while block
// row K is computed, so the chain of dependent block rows pays the memory
// latency once instead of once per row.  Requires bl, bu <= 16.
// ----------------------------------------------------------------------
constexpr int CS_B = 16;
__global__ __launch_bounds__(1024) void k_coarse_solve(const double *__restrict__ F, const SubInfo *__restrict__ sp,
                                                       const double *__restrict__ r, double *__restrict__ z,
                                                       double *__restrict__ ybuf) {
  constexpr int T = 32, G = 32;
  __shared__ double ring[RING][T];
  __shared__ double acc_s[T];
  const SubInfo s = *sp;
  const int tid = threadIdx.x, i = tid / G, g = tid % G;
  const int W = s.bl + s.bu + 1;
  auto at = [&](int K, int slot) -> const double * { return F + s.base + ((int64_t)K * W + slot) * (T * T) + i * T + g; };
  double cur[CS_B + 1], nxt[CS_B + 1];
  // forward: off-diagonal tiles of block row K are slots t = 0..bl-1 (P = K - bl + t)
  auto load_fwd = [&](int K, double (&b)[CS_B + 1]) {
#pragma unroll
    for (int t = 0; t < CS_B; ++t)
      if (t < s.bl && K - s.bl + t >= 0) b[t] = *at(K, t);
    b[CS_B] = *at(K, s.bl);
  };
  load_fwd(0, cur);
  for (int K = 0; K < s.nt; ++K) {
    const double bv = (g == 0 && K * T + i < s.n_loc) ? r[K * T + i] : 0.0;
    if (K + 1 < s.nt) load_fwd(K + 1, nxt);
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < CS_B; ++t)
      if (t < s.bl && K - s.bl + t >= 0) a += cur[t] * ring[(K - s.bl + t) % RING][g];
    a = group_sum<G>(a);
    if (g == 0) acc_s[i] = bv - a;
    lds_barrier();
    double y = (g < i) ? cur[CS_B] * acc_s[g] : 0.0;
    y = group_sum<G>(y);
    if (g == 0) {
      const double v = acc_s[i] + y;
      ring[K % RING][i] = v;
      if (K * T + i < s.n_loc) ybuf[K * T + i] = v;
    }
    lds_barrier();
#pragma unroll
    for (int t = 0; t <= CS_B; ++t) cur[t] = nxt[t];
  }
  // backward: off-diagonal tiles of block row K are slots bl+1+t (J = K + 1 + t)
  auto load_bwd = [&](int K, double (&b)[CS_B + 1]) {
#pragma unroll
    for (int t = 0; t < CS_B; ++t)
      if (t < s.bu && K + 1 + t < s.nt) b[t] = *at(K, s.bl + 1 + t);
    b[CS_B] = *at(K, s.bl);
  };
  load_bwd(s.nt - 1, cur);
  for (int K = s.nt - 1; K >= 0; --K) {
    const double bv = (g == 0 && K * T + i < s.n_loc) ? ybuf[K * T + i] : 0.0;
    if (K > 0) load_bwd(K - 1, nxt);
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < CS_B; ++t)
      if (t < s.bu && K + 1 + t < s.nt) a += cur[t] * ring[(K + 1 + t) % RING][g];
    a = group_sum<G>(a);
    if (g == 0) acc_s[i] = bv - a;
    lds_barrier();
    double y = (g >= i) ? cur[CS_B] * acc_s[g] : 0.0;
    y = group_sum<G>(y);
    if (g == 0) {
      ring[K % RING][i] = y;
      if (K * T + i < s.n_loc) z[K * T + i] = y;
    }
    lds_barrier();
#pragma unroll
    for (int t = 0; t <= CS_B; ++t) cur[t] = nxt[t];
  }
}

void launch_coarse_solve(const double *F, const SubInfo *sp, const double *r, double *z, double *ybuf,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_solve, dim3(1), dim3(1024), 0, st, F, sp, r, z, ybuf);
}

// ----------------------------------------------------------------------
// Explicit inverses of the coarse block-triangular factors.  With A_c =
// L U in tile-band storage (L block unit-lower: diagonal tiles L_KK unit
// lower, whose inverse's strict lower part is stored in the diagonal tile;
// U block upper: the diagonal tile's upper part holds U_KK^{-1}), tile
// column c of X = L^{-1} satisfies
//   X_cc = L_cc^{-1},   X_Kc = -L_KK^{-1} sum_{P=max(c,K-bl)}^{K-1} L_KP X_Pc  (K > c)
// and tile column c of W = U^{-1}
//   W_cc = U_cc^{-1},   W_Kc = -U_KK^{-1} sum_{J=K+1}^{min(c,K+bu)} U_KJ W_Jc  (K < c).
// Only the diagonal super-blocks of X and W are formed: tile rows are cut
// into blocks of S (the last one shorter), and the recurrences above run
// inside a block (X_II = L_II^{-1}, W_II = U_II^{-1}), so no column chain is
// longer than S.  With S >= bl, bu the factors couple only neighbouring
// blocks, and the coarse solve is a block sweep: forward y_I = X_II (r_I -
// L_{I,I-1} y_{I-1}), backward x_I = W_II (y_I - U_{I,I+1} x_{I+1}), each
// step a dense triangular mat-vec over the block plus a small coupling
// update; S = nt is the full inverse and the solve two mat-vecs.
//
// Packed tile storage, row-major 32x32 tiles, block after block (every
// earlier block holding S(S+1)/2 tiles): inside a block of nb rows, X tile
// (K, c), c <= K, at K(K+1)/2 + c; W tile (K, c), c >= K, at
// K nb - K(K-1)/2 + (c - K) (block-local indices).  A tile row is
// contiguous.
// ----------------------------------------------------------------------
__host__ __device__ inline int64_t lower_packed(int K, int c) { return (int64_t)K * (K + 1) / 2 + c; }
__host__ __device__ inline int64_t upper_packed(int K, int c, int nt) {
  return (int64_t)K * nt - (int64_t)K * (K - 1) / 2 + (c - K);
}

constexpr int INV_PF = 1;  // tile pairs loaded ahead into registers

// One launch forms both inverses: block b handles tile column b / 2 of X
// (even b) or column nt - 1 - b / 2 of W (odd b), so the longest columns
// of both start first.  Each of the four waves owns one 16x16 quadrant of
// the output tile and accumulates it on FP64 MFMA; one factor/inverse tile
// pair at a time is staged in LDS (17 KB, which fits beside a
// subdomain-factorisation workgroup), with the next INV_PF pairs' loads in
// flight in registers.
__global__ __launch_bounds__(256) void k_coarse_tri_inverse(const double *__restrict__ F, SubInfo s, int S,
                                                            double *__restrict__ X, double *__restrict__ Wm) {
  constexpr int T = 32;
  typedef Mfma<double>::v4 v4;
  __shared__ double As[T][T + 1];
  __shared__ double Bs[T][T + 1];
  const int nt = s.nt;
  const bool upper = (blockIdx.x & 1) != 0;
  const int c = upper ? nt - 1 - (int)(blockIdx.x >> 1) : (int)(blockIdx.x >> 1);
  double *const M = upper ? Wm : X;
  // the diagonal super-block of tile rows s0 .. s1 - 1 that holds column c,
  // and the packed storage of its inverse (every earlier block has S rows)
  const int sb = c / S, s0 = sb * S, s1 = min(s0 + S, nt), nb = s1 - s0;
  const int64_t boff = (int64_t)sb * S * (S + 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int qi = wave >> 1, qj = wave & 1;
  const int W = s.bl + s.bu + 1;
  auto fac = [&](int K, int slot) { return F + s.base + ((int64_t)K * W + slot) * (T * T); };
  auto out = [&](int K) -> double * {
    return M + (boff + (upper ? upper_packed(K - s0, c - s0, nb) : lower_packed(K - s0, c - s0))) * (T * T);
  };
  const int rows = upper ? c - s0 + 1 : s1 - c;
  for (int it = 0; it < rows; ++it) {
    const int K = upper ? c - it : c + it;
    const int p_lo = upper ? K + 1 : max(c, K - s.bl);
    const int p_hi = upper ? min(c, K + s.bu) : K - 1;
    v4 acc = {0.0, 0.0, 0.0, 0.0};
    double ca[INV_PF][4], cb[INV_PF][4];
    auto load_group = [&](int P0, double (&ga)[INV_PF][4], double (&gb)[INV_PF][4]) {
#pragma unroll
      for (int q = 0; q < INV_PF; ++q)
        if (P0 + q <= p_hi) {
          const double *a = fac(K, P0 + q - K + s.bl);
          const double *b = out(P0 + q);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            ga[q][m] = a[tid + 256 * m];
            gb[q][m] = b[tid + 256 * m];
          }
        }
    };
    load_group(p_lo, ca, cb);
    for (int P0 = p_lo; P0 <= p_hi; P0 += INV_PF) {
      double na[INV_PF][4], nb[INV_PF][4];
      load_group(P0 + INV_PF, na, nb);
#pragma unroll
      for (int q = 0; q < INV_PF; ++q)
        if (P0 + q <= p_hi) {
          __syncthreads();  // the previous pair is consumed
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int e = tid + 256 * m;
            As[e / T][e % T] = ca[q][m];
            Bs[e / T][e % T] = cb[q][m];
          }
          __syncthreads();
#pragma unroll
          for (int k0 = 0; k0 < T; k0 += 4)
            acc = Mfma<double>::op(As[16 * qi + lr][k0 + lk], Bs[k0 + lk][16 * qj + lr], acc);
        }
#pragma unroll
      for (int q = 0; q < INV_PF; ++q)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          ca[q][m] = na[q][m];
          cb[q][m] = nb[q][m];
        }
    }
    __syncthreads();
    // S (the sum, or -I on the diagonal so that the diagonal tile is -D (-I))
    // into Bs; D = L_KK^{-1} (unit lower) or U_KK^{-1} (upper) into As
    const double *d = fac(K, s.bl);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * qi + Mfma<double>::row(lk, v), j = 16 * qj + lr;
      Bs[i][j] = K == c ? (i == j ? -1.0 : 0.0) : acc[v];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = tid + 256 * m, i = e / T, j = e % T;
      const double dv = d[e];
      As[i][j] = upper ? (j >= i ? dv : 0.0) : (j < i ? dv : (i == j ? 1.0 : 0.0));
    }
    __syncthreads();
    v4 r = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < T; k0 += 4) r = Mfma<double>::op(As[16 * qi + lr][k0 + lk], Bs[k0 + lk][16 * qj + lr], r);
    double *o = out(K);
#pragma unroll
    for (int v = 0; v < 4; ++v) o[(16 * qi + Mfma<double>::row(lk, v)) * T + 16 * qj + lr] = -r[v];
    // the next rows read this tile back through the cache: make the stores
    // visible to the whole workgroup
    __threadfence_block();
    __syncthreads();
  }
}

// y = M x for a packed triangular tile matrix M (X: lower, W: upper), or
// y = M^T x (TRANS), in two launches.  The tile rows of M (the tile columns
// when transposed) are cut into chunks of TRI_CW tiles, one workgroup per
// chunk, so that the longest rows no longer set the time of the launch;
// each chunk writes its partial sums, and a second launch adds a row's
// partials in chunk order (fixed order, so results are reproducible).
// Row K (0-based in the block of nt rows) holds len(K) tiles: K + 1 when
// the stored rows grow (lower non-transposed, upper transposed), else
// nt - K.  Chunks are numbered row by row: row K's first chunk is
// before(K) = C(K) (growing) or C(nt) - C(nt - K), with C(n) the sum of
// ceil(m / TRI_CW) over m = 1 .. n; C(nt) chunks in all.
constexpr int TRI_CW = 8;
__host__ __device__ inline int64_t tri_csum(int n) {
  const int64_t q = n / TRI_CW, r = n % TRI_CW;
  return n + TRI_CW * q * (q - 1) / 2 + r * q;
}
__host__ __device__ inline int64_t tri_before(int K, int nt, bool grows) {
  return grows ? tri_csum(K) : tri_csum(nt) - tri_csum(nt - K);
}
int64_t coarse_tri_chunks(int nt) { return tri_csum(nt); }

template <bool UPPER, bool TRANS>
__global__ __launch_bounds__(256) void k_coarse_tri_gemv(const double *__restrict__ M, int nt,
                                                         const double *__restrict__ x, double *__restrict__ part) {
  constexpr int T = 32;
  __shared__ double red[8][T];
  const int tid = threadIdx.x;
  const bool grows = (!UPPER) != TRANS;
  // the chunk's row: the last K with before(K) <= chunk (uniform search)
  const int64_t b = blockIdx.x;
  int lo = 0, hi = nt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tri_before(mid, nt, grows) <= b) lo = mid;
    else hi = mid - 1;
  }
  const int K = lo;
  const int c = (int)(b - tri_before(K, nt, grows));
  const int r_lo = grows ? 0 : K, r_hi = grows ? K : nt - 1;
  const int c_lo = r_lo + c * TRI_CW, c_hi = min(r_hi, c_lo + TRI_CW - 1);
  auto tile = [&](int cc) -> const double * {
    // tile (row, col) of M: M_K,cc, or M_cc,K when transposed
    const int r0 = TRANS ? cc : K, c0 = TRANS ? K : cc;
    return M + (UPPER ? upper_packed(r0, c0, nt) : lower_packed(r0, c0)) * (T * T);
  };
  double acc = 0.0;
  if constexpr (!TRANS) {
    const int i = tid >> 3, g = tid & 7;
    int cc = c_lo;
    for (; cc + 3 <= c_hi; cc += 4) {
      double4 a4[4], b4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a4[u] = *reinterpret_cast<const double4 *>(tile(cc + u) + i * T + 4 * g);
        b4[u] = *reinterpret_cast<const double4 *>(x + (int64_t)(cc + u) * T + 4 * g);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc += a4[u].x * b4[u].x + a4[u].y * b4[u].y + a4[u].z * b4[u].z + a4[u].w * b4[u].w;
    }
    for (; cc <= c_hi; ++cc) {
      const double4 a4 = *reinterpret_cast<const double4 *>(tile(cc) + i * T + 4 * g);
      const double4 b4 = *reinterpret_cast<const double4 *>(x + (int64_t)cc * T + 4 * g);
      acc += a4.x * b4.x + a4.y * b4.y + a4.z * b4.z + a4.w * b4.w;
    }
    // sum the 8 column groups of row i (consecutive lanes)
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) acc += __shfl_xor(acc, o, 8);
    if (g == 0) part[b * T + i] = acc;
  } else {
    const int j = tid & 31, g = tid >> 5;  // rows 4g .. 4g+3 of each tile
    int cc = c_lo;
    for (; cc + 1 <= c_hi; cc += 2) {
      double a2[2][4], b2[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          a2[u][m] = tile(cc + u)[(4 * g + m) * T + j];
          b2[u][m] = x[(int64_t)(cc + u) * T + 4 * g + m];
        }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc += a2[u][m] * b2[u][m];
    }
    for (; cc <= c_hi; ++cc)
#pragma unroll
      for (int m = 0; m < 4; ++m) acc += tile(cc)[(4 * g + m) * T + j] * x[(int64_t)cc * T + 4 * g + m];
    red[g][j] = acc;
    __syncthreads();
    if (tid < T) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += red[q][tid];
      part[b * T + tid] = t;
    }
  }
}

// y_K = sum of row K's chunk partials, in chunk order (one workgroup of T
// threads per row)
__global__ __launch_bounds__(32) void k_coarse_tri_reduce(const double *__restrict__ part, int nt, int grows,
                                                          double *__restrict__ y) {
  constexpr int T = 32;
  const int K = blockIdx.x, i = threadIdx.x;
  const int64_t b0 = tri_before(K, nt, grows), b1 = tri_before(K + 1, nt, grows);
  double t = 0.0;
  for (int64_t b = b0; b < b1; ++b) t += part[b * T + i];
  y[(int64_t)K * T + i] = t;
}

// Coupling step of the coarse block sweep: v_K -= (tiles of row K of the
// factor that lie in the neighbouring block) x (that block's solution sol).
//   L (forward):      K in [s0, s0 + bl),  v_K -= sum_{P = K-bl}^{s0-1} L_KP sol_P
//   U (backward):     K in [s1 - bu, s1),  v_K -= sum_{J = s1}^{K+bu} U_KJ sol_J
//   U^T (forward):    K in [s0, s0 + bu),  v_K -= sum_{P = K-bu}^{s0-1} U_PK^T sol_P
//   L^T (backward):   K in [s1 - bl, s1),  v_K -= sum_{J = s1}^{K+bl} L_JK^T sol_J
// for the block of tile rows s0 .. s1 - 1.  One workgroup per tile row K.
template <bool UPPER, bool TRANS>
__global__ __launch_bounds__(256) void k_coarse_couple(const double *__restrict__ F, SubInfo s, int S, int sb,
                                                       double *__restrict__ v, const double *__restrict__ sol) {
  constexpr int T = 32;
  __shared__ double red[8][T];
  const int nt = s.nt, s0 = sb * S, s1 = min(s0 + S, nt);
  constexpr bool fwd = UPPER == TRANS;
  const int w = UPPER ? s.bu : s.bl;
  const int K = fwd ? s0 + (int)blockIdx.x : s1 - 1 - (int)blockIdx.x;
  if (fwd ? (K >= min(s0 + w, s1)) : (K < max(s1 - w, s0))) return;  // uniform per workgroup
  const int lo = fwd ? max(K - w, 0) : s1, hi = fwd ? s0 - 1 : min(K + w, nt - 1);
  const int Wd = s.bl + s.bu + 1;
  auto tile = [&](int r, int c) { return F + s.base + ((int64_t)r * Wd + (c - r + s.bl)) * (T * T); };
  const int tid = threadIdx.x;
  double acc = 0.0;
  if constexpr (!TRANS) {
    const int i = tid >> 3, g = tid & 7;
    for (int c = lo; c <= hi; ++c) {
      const double4 a = *reinterpret_cast<const double4 *>(tile(K, c) + i * T + 4 * g);
      const double4 b = *reinterpret_cast<const double4 *>(sol + (int64_t)c * T + 4 * g);
      acc += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) acc += __shfl_xor(acc, o, 8);
    if (g == 0) v[(int64_t)K * T + i] -= acc;
  } else {
    const int j = tid & 31, g = tid >> 5;  // rows 4g .. 4g+3 of each tile
    for (int c = lo; c <= hi; ++c) {
      const double *a = tile(c, K);
#pragma unroll
      for (int m = 0; m < 4; ++m) acc += a[(4 * g + m) * T + j] * sol[(int64_t)c * T + 4 * g + m];
    }
    red[g][j] = acc;
    __syncthreads();
    if (tid < T) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += red[q][tid];
      v[(int64_t)K * T + tid] -= t;
    }
  }
}

void launch_coarse_inverse(const double *F, const SubInfo &cs, int S, double *X, double *W, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_tri_inverse, dim3(2 * cs.nt), dim3(256), 0, st, F, cs, S, X, W);
}

void launch_coarse_inverse_apply(const double *X, const double *W, const double *F, const SubInfo &cs, int S,
                                 double *r, double *z, double *tmp, double *part, int transpose, hipStream_t st) {
  constexpr int T = 32;
  const int nt = cs.nt, NS = (nt + S - 1) / S;
  auto gemv = [&](auto kern, bool grows, const double *M, int sb, const double *x, double *y) {
    const int s0 = sb * S, nb = std::min(S, nt - s0);
    const int64_t off = (int64_t)sb * S * (S + 1) / 2 * (T * T);
    hipLaunchKernelGGL(kern, dim3((unsigned)tri_csum(nb)), dim3(256), 0, st, M + off, nb, x + (int64_t)s0 * T, part);
    hipLaunchKernelGGL(k_coarse_tri_reduce, dim3(nb), dim3(T), 0, st, part, nb, (int)grows, y + (int64_t)s0 * T);
  };
  if (!transpose) {  // L y = r (y in tmp) forward, then U z = y backward
    for (int sb = 0; sb < NS; ++sb) {
      if (sb > 0)
        hipLaunchKernelGGL((k_coarse_couple<false, false>), dim3(cs.bl), dim3(256), 0, st, F, cs, S, sb, r, tmp);
      gemv(k_coarse_tri_gemv<false, false>, true, X, sb, r, tmp);
    }
    for (int sb = NS - 1; sb >= 0; --sb) {
      if (sb < NS - 1)
        hipLaunchKernelGGL((k_coarse_couple<true, false>), dim3(cs.bu), dim3(256), 0, st, F, cs, S, sb, tmp, z);
      gemv(k_coarse_tri_gemv<true, false>, false, W, sb, tmp, z);
    }
  } else {  // U^T y = r forward, then L^T z = y backward
    for (int sb = 0; sb < NS; ++sb) {
      if (sb > 0)
        hipLaunchKernelGGL((k_coarse_couple<true, true>), dim3(cs.bu), dim3(256), 0, st, F, cs, S, sb, r, tmp);
      gemv(k_coarse_tri_gemv<true, true>, true, W, sb, r, tmp);
    }
    for (int sb = NS - 1; sb >= 0; --sb) {
      if (sb < NS - 1)
        hipLaunchKernelGGL((k_coarse_couple<false, true>), dim3(cs.bl), dim3(256), 0, st, F, cs, S, sb, tmp, z);
      gemv(k_coarse_tri_gemv<false, true>, false, X, sb, tmp, z);
    }
  }
}

// ----------------------------------------------------------------------
// Discrete adjoint support (counts, adjoint right-hand side, parameter
// gradients).  With lam^n the adjoint state of step n:
//   rhs = dJ/du^n + M lam^{n+1},  dJ/dc_r^n = gc[r],  c_r = sum_{j in r} m_j i_j
//   grad_g[j] -= (lam_S - lam_E)_j dt m_j a_j (beta_I i_j + beta_E e_j) s_j
//   grad_nu[c] -= dt sum_i lam_{c,i} sum_T Nbar_T sum_k K^T_ik u_{c,k}
// ----------------------------------------------------------------------
// counts[r] = sum over the nodes of region r (CSR reg_ptr/reg_nodes) of m_j i_j
__global__ __launch_bounds__(256) void k_region_counts(const int64_t *__restrict__ reg_ptr,
                                                       const int32_t *__restrict__ reg_nodes,
                                                       const double *__restrict__ mass, const double *__restrict__ u,
                                                       double *__restrict__ counts) {
  __shared__ double lds4[4];
  const int r = blockIdx.x;
  double a = 0.0;
  for (int64_t k = reg_ptr[r] + threadIdx.x; k < reg_ptr[r + 1]; k += 256) {
    const int64_t j = reg_nodes[k];
    a += mass[j] * u[5 * j + 2];
  }
  const double t = block_sum(a, lds4);
  if (threadIdx.x == 0) counts[r] = t;
}

// rhs = M^T lam^{n+1} + dL/du^n (the observation weights the infected
// compartment by the lumped mass); M^T = M for the lumped and the
// consistent mass
__global__ __launch_bounds__(256) void k_adjoint_rhs(MeshDev md, const int32_t *__restrict__ region,
                                                     const double *__restrict__ gc, const double *__restrict__ lam_next,
                                                     double *__restrict__ rhs) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= md.n) return;
  const double m = md.mass[j];
  double v[5];
  if (md.cmass_d) {
    const double d = md.cmass_d[j];
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = d * lam_next[5 * j + c];
    for (int64_t s = md.rowptr[j]; s < md.rowptr[j + 1]; ++s) {
      const int64_t k = md.col[s];
      const double o = md.cmass_o[s];
#pragma unroll
      for (int c = 0; c < 5; ++c) v[c] += o * lam_next[5 * k + c];
    }
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = m * lam_next[5 * j + c];
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) rhs[5 * j + c] = v[c];
  const int32_t r = region[j];
  if (r >= 0) rhs[5 * j + 2] += gc[r] * m;
}

// gradient contributions of one step; nu partial sums per block in
// partials[c * nb + block]
__global__ __launch_bounds__(256) void k_adjoint_grad(MeshDev m, ParamsDev P0, const double *__restrict__ u,
                                                      const double *__restrict__ lam, double dt,
                                                      double *__restrict__ grad_g, double *__restrict__ partials) {
  __shared__ double lds4[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double pc[5] = {0, 0, 0, 0, 0};
  if (i < m.n) {
    const ParamsDev P = m.inst ? m.Pinst[m.inst[i]] : P0;
    double ui[5];
    load5(u + 5 * i, ui);
    const double Ni = ui[0] + ui[1] + ui[2] + ui[3] + ui[4];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t k = m.inc_ptr[i]; k < m.inc_ptr[i + 1]; ++k) {
      const int32_t j = m.inc_j[k], l = m.inc_l[k];
      const double Kii = m.inc_K[3 * k], Kij = m.inc_K[3 * k + 1], Kil = m.inc_K[3 * k + 2];
      double uj[5], ul[5];
      load5(u + 5 * (int64_t)j, uj);
      load5(u + 5 * (int64_t)l, ul);
      const double Nbar = (Ni + (uj[0] + uj[1] + uj[2] + uj[3] + uj[4]) + (ul[0] + ul[1] + ul[2] + ul[3] + ul[4])) *
                          (1.0 / 3.0);
#pragma unroll
      for (int c = 0; c < 5; ++c) acc[c] += Nbar * (Kii * ui[c] + Kij * uj[c] + Kil * ul[c]);
    }
    double li[5];
    load5(lam + 5 * i, li);
#pragma unroll
    for (int c = 0; c < 5; ++c) pc[c] = li[c] * acc[c];
    const double a = 1.0 - P.A / Ni;
    const double dFs = dt * m.mass[i] * a * (P.bI * ui[2] + P.bE * ui[1]) * ui[0];
    grad_g[i] -= (li[0] - li[1]) * dFs;
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double t = block_sum(pc[c], lds4);
    if (threadIdx.x == 0) partials[(int64_t)c * gridDim.x + blockIdx.x] = t;
  }
}

void launch_region_counts(const int64_t *reg_ptr, const int32_t *reg_nodes, const double *mass, const double *u,
                          double *counts, int n_regions, hipStream_t st) {
  if (n_regions > 0)
    hipLaunchKernelGGL(k_region_counts, dim3(n_regions), dim3(256), 0, st, reg_ptr, reg_nodes, mass, u, counts);
}
void launch_adjoint_rhs(const MeshDev &m, const int32_t *region, const double *gc, const double *lam_next,
                        double *rhs, hipStream_t st) {
  const int64_t n = m.n;
  hipLaunchKernelGGL(k_adjoint_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, region, gc, lam_next,
                     rhs);
}
int launch_adjoint_grad(const MeshDev &m, const ParamsDev &P, const double *u, const double *lam, double dt,
                        double *grad_g, double *partials, hipStream_t st) {
  const unsigned nb = (unsigned)((m.n + 255) / 256);
  hipLaunchKernelGGL(k_adjoint_grad, dim3(nb), dim3(256), 0, st, m, P, u, lam, dt, grad_g, partials);
  return (int)nb;
}

// ----------------------------------------------------------------------
// launchers

void launch_seg_mdot(const SegHost &g, const double *V, int64_t ldv, int nv, const double *w, int with_self,
                     double *partials, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_mdot<KRYLOV_MAX>, dim3(g.B), dim3(256), 0, st, g.view(), V, ldv, nv, w, with_self,
                     partials);
}
void launch_seg_reduce(const SegHost &g, const double *partials, int nrows, double *out, int ldo, int row_off,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_seg_reduce, dim3(g.S * nrows), dim3(256), 0, st, g.view(), partials, nrows, out, ldo, row_off);
}
void launch_seg_maxpy_norm(const SegHost &g, double *w, const double *V, int64_t ldv, const double *h, int ldh, int nv,
                           double *partials, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_maxpy_norm<KRYLOV_MAX>, dim3(g.B), dim3(256), 0, st, g.view(), w, V, ldv, h, ldh, nv,
                     partials);
}
void launch_seg_gemv_update(const SegHost &g, double *x, const double *Z, int64_t ldz, const double *y, int ldy, int nv,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_seg_gemv_update<KRYLOV_MAX>, dim3(g.B), dim3(256), 0, st, g.view(), x, Z, ldz, y, ldy, nv);
}
void launch_seg_axpby(const SegHost &g, double *y, const double *x, const double *a, double b, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_axpby, dim3(g.B), dim3(256), 0, st, g.view(), y, x, a, b);
}
void launch_seg_norm2(const SegHost &g, const double *x, const double *scale, double *partials, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_norm2, dim3(g.B), dim3(256), 0, st, g.view(), x, scale, partials);
}
// ----------------------------------------------------------------------
static inline unsigned nblocks(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

void launch_residual(const MeshDev &m, const ParamsDev &P, const double *g, const double *u, const double *up,
                     double dt, const double *src, double *F, hipStream_t st) {
  hipLaunchKernelGGL(k_residual, dim3(nblocks(m.n)), dim3(256), 0, st, m, P, g, u, up, dt, src, F);
}
void launch_jacobian(const MeshDev &m, const ParamsDev &P, const double *g, const double *u, double dt, double *diag,
                     double *off, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobian, dim3(nblocks(m.n)), dim3(256), 0, st, m, P, g, u, dt, diag);
  if (m.nslots > 0)
    hipLaunchKernelGGL(k_jacobian_off, dim3(nblocks(m.nslots)), dim3(256), 0, st, m, P, u, dt, off);
}
void launch_spmv(const MeshDev &m, const double *diag, const double *off, const double *x, const double *b, double *y,
                 int transpose, hipStream_t st) {
  if (transpose)
    hipLaunchKernelGGL(k_spmv_t, dim3(nblocks(m.n, 4 * SPMV_WAVE_NODES)), dim3(256), 0, st, m, diag, off, x, b, y);
  else
    hipLaunchKernelGGL(k_spmv, dim3(nblocks(m.n, 4 * SPMV_WAVE_NODES)), dim3(256), 0, st, m, diag, off, x, b, y);
}
void launch_mdot(const double *V, int64_t ldv, int nv, const double *w, int64_t N, int with_self, double *partials,
                 int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_mdot<KRYLOV_MAX>, dim3(nb), dim3(256), 0, st, V, ldv, nv, w, N, with_self, partials);
}
void launch_reduce(const double *partials, int nb, int nv, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(nv), dim3(256), 0, st, partials, nb, out);
}
void launch_maxpy_norm(double *w, const double *V, int64_t ldv, const double *h, int nv, int64_t N, double *partials,
                       int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_maxpy_norm<KRYLOV_MAX>, dim3(nb), dim3(256), 0, st, w, V, ldv, h, nv, N, partials);
}
void launch_gemv_update(double *x, const double *Z, int64_t ldz, const double *y, int nv, int64_t N, int nb,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_update<KRYLOV_MAX>, dim3(nb), dim3(256), 0, st, x, Z, ldz, y, nv, N);
}
void launch_axpby(double *y, const double *x, double a, const double *aptr, int ainv, double b, int64_t N, int nb,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(nb), dim3(256), 0, st, y, x, a, aptr, ainv, b, N);
}
void launch_norm2_partials(const double *x, const double *scale, int64_t N, double *partials, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2_partials, dim3(nb), dim3(256), 0, st, x, scale, N, partials);
}
void launch_csr_values(const MeshDev &m, const double *diag, const double *off, const int64_t *csr_rowptr,
                       double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_csr_values, dim3(nblocks(5 * m.n)), dim3(256), 0, st, m, diag, off, csr_rowptr, out);
}
void launch_pgs_stiffness(const MeshDev &m, const double *uk, double *Kd, double *Ko, hipStream_t st) {
  hipLaunchKernelGGL(k_pgs_stiffness, dim3(nblocks(m.n)), dim3(256), 0, st, m, uk, Kd, Ko);
}
void launch_pgs_system(const MeshDev &m, const ParamsDev &P, const double *g, int c, double dt, const double *u,
                       const double *uk, const double *un, const double *Kd, const double *Ko, double *sdiag,
                       double *soff, double *r, hipStream_t st) {
  hipLaunchKernelGGL(k_pgs_system, dim3(nblocks(m.n)), dim3(256), 0, st, m, P, g, c, dt, u, uk, un, Kd, Ko, sdiag,
                     soff, r);
}
void launch_scalar_spmv(const MeshDev &m, const double *sdiag, const double *soff, const double *x, const double *b,
                        double *y, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_spmv, dim3(nblocks(m.n)), dim3(256), 0, st, m, sdiag, soff, x, b, y);
}
void launch_pgs_update(double *u, int c, const double *delta, const double *sdiag, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_pgs_update, dim3(nblocks(n)), dim3(256), 0, st, u, c, delta, sdiag, n);
}

void launch_check_state(const double *u, int64_t n, const int32_t *inst, int *flags, hipStream_t st) {
  hipLaunchKernelGGL(k_check_state, dim3(nblocks(n)), dim3(256), 0, st, u, n, inst, flags);
}

template <int T, class ET>
static void extract_t(const FactorLaunch &fl, ET *F, const double *diag, const double *off, hipStream_t st) {
  if (fl.ntrows <= 0) return;
  // a register slot per node block: 10 covers P1 meshes of node degree <= 9
  const dim3 g((unsigned)fl.ntrows);
  if (fl.bs == 1) {
    if (fl.max_node_blocks <= 10)
      hipLaunchKernelGGL((k_extract_tiles<T, ET, 10, 1>), g, dim3(256), 0, st, F, fl.subs, fl.trow_ptr, fl.trow_sub,
                         fl.erow, fl.elo, fl.ent, fl.ent_ptr, diag, off);
    else
      hipLaunchKernelGGL((k_extract_tiles<T, ET, 16, 1>), g, dim3(256), 0, st, F, fl.subs, fl.trow_ptr, fl.trow_sub,
                         fl.erow, fl.elo, fl.ent, fl.ent_ptr, diag, off);
  } else if (fl.dense_off) {
    hipLaunchKernelGGL((k_extract_tiles<T, ET, 16, 5, true>), g, dim3(256), 0, st, F, fl.subs, fl.trow_ptr,
                       fl.trow_sub, fl.erow, fl.elo, fl.ent, fl.ent_ptr, diag, off);
  } else if (fl.max_node_blocks <= 10) {
    hipLaunchKernelGGL((k_extract_tiles<T, ET, 10>), g, dim3(256), 0, st, F, fl.subs, fl.trow_ptr, fl.trow_sub,
                       fl.erow, fl.elo, fl.ent, fl.ent_ptr, diag, off);
  } else {
    hipLaunchKernelGGL((k_extract_tiles<T, ET, 16>), g, dim3(256), 0, st, F, fl.subs, fl.trow_ptr, fl.trow_sub,
                       fl.erow, fl.elo, fl.ent, fl.ent_ptr, diag, off);
  }
}

template <int T>
static void coarse_factor_t(const FactorLaunch &fl, const double *diag, const double *off, hipStream_t st) {
  HIPCHECK(hipMemsetAsync(fl.Fc, 0, sizeof(double) * fl.coarse_entries, st));
  hipLaunchKernelGGL((k_pad_identity<T, double>), dim3(1), dim3(256), 0, st, fl.Fc, fl.coarse_dev, nullptr, nullptr,
                     1);
  hipLaunchKernelGGL(k_galerkin<T>, dim3(nblocks(fl.gal_nblk * 64)), dim3(256), 0, st, fl.Fc, fl.cs, fl.gp, fl.gq,
                     fl.gptr, fl.gref, fl.gw, fl.gal_nblk, diag, off, fl.status);
  const SubInfo cs = fl.cs;
  if constexpr (T == 32) {
    hipLaunchKernelGGL(k_lu_step_diag<T>, dim3(1), dim3(256), 0, st, fl.Fc, cs, 0, fl.status);
    for (int K = 0; K < cs.nt; ++K)
      hipLaunchKernelGGL(k_lu_step_fused, dim3(cs.bl * cs.bu + cs.bl + cs.bu), dim3(256), 0, st, fl.Fc, cs, K,
                         fl.status);
  } else {
    for (int K = 0; K < cs.nt; ++K) {
      hipLaunchKernelGGL(k_lu_step_diag<T>, dim3(1), dim3(256), 0, st, fl.Fc, cs, K, fl.status);
      if (K + 1 < cs.nt) {
        hipLaunchKernelGGL(k_lu_step_panel<T>, dim3(cs.bl + cs.bu), dim3(256), 0, st, fl.Fc, cs, K);
        hipLaunchKernelGGL(k_lu_step_schur<T>, dim3(cs.bl * cs.bu), dim3(256), 0, st, fl.Fc, cs, K);
      }
    }
  }
}

// Subdomain factorisation launch (waves x panel tiles per wave): 4 x 2 when
// every U panel fits; else 8 x 2, except float32 beside a coarse chain,
// where 4 x 3 (two workgroups of 220 VGPRs per compute unit) leaves the
// 64 VGPRs per SIMD lane that the coarse kernels need, while two 8 x 2
// workgroups of 128 would fill the register file.
template <class CT>
static void band_lu32(const FactorLaunch &fl, CT *F, hipStream_t st) {
  if (sizeof(CT) == 4) {
    // float32: four waves with three panel tiles each, two workgroups per
    // compute unit with room left for the float64 coarse-chain kernels
    if (fl.Fh)
      hipLaunchKernelGGL((k_band_lu32<CT, 4, 3, true>), dim3(fl.nsub), dim3(256), 0, st, F, fl.subs, fl.erow,
                         fl.elo, fl.order, fl.nsub, nullptr, fl.status, (__hip_bfloat16 *)fl.Fh);
    else
      hipLaunchKernelGGL((k_band_lu32<CT, 4, 3, false>), dim3(fl.nsub), dim3(256), 0, st, F, fl.subs, fl.erow,
                         fl.elo, fl.order, fl.nsub, nullptr, fl.status, (__hip_bfloat16 *)nullptr);
    return;
  }
  // float64: two workgroups of four waves per compute unit.  Beside a
  // coarse chain (its kernels need 64 registers per lane), a persistent
  // grid of 2 CUs - lu_spare workgroups draws the subdomains from a queue,
  // so that some compute units keep room for the chain.
  const int per_cu = 2;
  int grid = fl.nsub;
  int *queue = nullptr;
  if (fl.coarse && fl.queue && fl.n_cu > 0) {
    grid = std::min(fl.nsub, std::max(1, per_cu * fl.n_cu - fl.lu_spare));
    if (grid < fl.nsub) {
      queue = fl.queue;
      hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, queue, grid, 1);
    }
  }
  hipLaunchKernelGGL((k_band_lu32<CT, 4, 2, false>), dim3(grid), dim3(256), 0, st, F, fl.subs, fl.erow, fl.elo,
                     fl.order, fl.nsub, queue, fl.status, (__hip_bfloat16 *)nullptr);
}

static void coarse_factor(const FactorLaunch &fl, const double *diag, const double *off, hipStream_t st) {
  if (fl.tile == 32)
    coarse_factor_t<32>(fl, diag, off, st);
  else
    coarse_factor_t<16>(fl, diag, off, st);
}

void launch_setup_factors(const FactorLaunch &fl, const double *diag, const double *off, hipStream_t st,
                          hipStream_t st_coarse) {
  // The two chains run side by side; the one on the critical path is queued
  // first, because the host spends a while queueing the coarse chain (one
  // launch per coarse tile row) and the device starts each chain as its
  // launches arrive.  Float64 subdomain factors take longer than the coarse
  // chain; with float32 factors the coarse chain is the longer one.
  const bool coarse_first = fl.coarse && fl.sub_float;
  if (coarse_first) coarse_factor(fl, diag, off, st_coarse);
  if (fl.nsub > 0) {
    auto mark = [&](hipEvent_t e) {
      if (e) HIPCHECK(hipEventRecord(e, st));
    };
    mark(fl.ev_extract);
    if (fl.tile == 32) {
      if (fl.sub_float) {
        extract_t<32, float>(fl, (float *)fl.Fs, diag, off, st);
        mark(fl.ev_lu);
        band_lu32<float>(fl, (float *)fl.Fs, st);
      } else {
        extract_t<32, double>(fl, (double *)fl.Fs, diag, off, st);
        mark(fl.ev_lu);
        band_lu32<double>(fl, (double *)fl.Fs, st);
      }
    } else {
      extract_t<16, double>(fl, (double *)fl.Fs, diag, off, st);
      mark(fl.ev_lu);
      const size_t lds = (size_t)std::max(fl.max_bu, 1) * 16 * 17 * sizeof(double);
      hipLaunchKernelGGL(k_band_lu<16>, dim3(fl.nsub), dim3(256), lds, st, (double *)fl.Fs, fl.subs, fl.erow, fl.elo,
                         fl.order, fl.status);
    }
    mark(fl.ev_lu_end);
  }
  if (fl.coarse && !coarse_first) coarse_factor(fl, diag, off, st_coarse);
}

void launch_galerkin_blocks(const int32_t *gdst, const int64_t *gptr, const int32_t *gref, const double *gw,
                            int64_t nblk, const double *diag, const double *off, double *cdiag, double *coff,
                            hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(k_galerkin_blocks<false>, dim3(nblocks(nblk * 64)), dim3(256), 0, st, cdiag, coff, gdst, gptr, gref, gw,
                     nblk, diag, off);
}

void launch_galerkin_dense(const int32_t *gdst, const int64_t *gptr, const int32_t *gref, int64_t nblk,
                           const double *diag, const double *off, double *cdiag, double *coff, hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(k_galerkin_blocks<true>, dim3(nblocks(nblk * 64)), dim3(256), 0, st, cdiag, coff, gdst, gptr,
                     gref, (const double *)nullptr, nblk, diag, off);
}
void launch_block_inv5(int64_t n, const double *diag, double *dinv, int *status, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_block_inv5, dim3(nblocks(n)), dim3(256), 0, st, n, diag, dinv, status);
}
void launch_block_jacobi(int64_t n, const double *dinv, const double *r, double omega, double *x, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_block_jacobi, dim3(nblocks(5 * n)), dim3(256), 0, st, n, dinv, r, omega, x);
}
void launch_agg_restrict(int64_t nagg, const int64_t *agg_ptr, const int32_t *agg_nodes, const double *r, double *bc,
                         hipStream_t st) {
  if (nagg > 0)
    hipLaunchKernelGGL(k_agg_restrict, dim3(nblocks(5 * nagg)), dim3(256), 0, st, nagg, agg_ptr, agg_nodes, r, bc);
}
void launch_agg_prolong(int64_t n, const int32_t *agg, const double *xc, double *x, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_agg_prolong, dim3(nblocks(5 * n)), dim3(256), 0, st, n, agg, xc, x);
}
void launch_dense_gemv(int m, const double *M, const double *b, double *y, hipStream_t st) {
  if (m > 0) hipLaunchKernelGGL(k_dense_gemv, dim3(nblocks(m)), dim3(256), 0, st, m, M, b, y);
}
void launch_block_spmv(int64_t n, const int64_t *rowptr, const int32_t *col, const double *diag, const double *off,
                       const double *x, const double *b, double *y, hipStream_t st) {
  if (n <= 0) return;
  const int64_t per_block = 4 * SPMV_WAVE_NODES;
  hipLaunchKernelGGL(k_block_spmv, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(256), 0, st, n, rowptr, col,
                     diag, off, x, b, y);
}

void launch_convert(void *dst, int dst_prec, const void *src, int src_float, int64_t N, hipStream_t st) {
  const unsigned nb = 4096;
  if (dst_prec == 1) {
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nb), dim3(256), 0, st, (float *)dst, (const double *)src, N);
  } else if (dst_prec == 2) {
    if (src_float)
      hipLaunchKernelGGL((k_convert<__hip_bfloat16, float>), dim3(nb), dim3(256), 0, st, (__hip_bfloat16 *)dst,
                         (const float *)src, N);
    else
      hipLaunchKernelGGL((k_convert<__hip_bfloat16, double>), dim3(nb), dim3(256), 0, st, (__hip_bfloat16 *)dst,
                         (const double *)src, N);
  }
}

template <int T, class FT, bool TR, int NTHR>
static void solve_launch(const SolveLaunch &sl, hipStream_t st) {
  hipLaunchKernelGGL((k_band_solve<T, FT, NTHR, TR>), dim3(sl.nblocks), dim3(NTHR), 0, st, (const FT *)sl.F, sl.subs,
                     sl.erow, sl.elo, sl.order, sl.l2g, sl.owned, sl.r, sl.z, sl.add, sl.yloc, sl.ybuf, sl.sub_seg,
                     sl.seg_active);
}
template <int T, class FT, bool TR>
static void solve_tt(const SolveLaunch &sl, hipStream_t st) {
  // wider forms need at least one tile element per lane: T = 32 only
  const int thr = sl.wide ? 1024 : sl.threads;
  if constexpr (T == 32) {
    if (thr == 1024) return solve_launch<T, FT, TR, 1024>(sl, st);
    if (thr == 512) return solve_launch<T, FT, TR, 512>(sl, st);
    if (thr == 128) return solve_launch<T, FT, TR, 128>(sl, st);
  }
  solve_launch<T, FT, TR, 256>(sl, st);
}
template <int T, class FT>
static void solve_t(const SolveLaunch &sl, hipStream_t st) {
  if (sl.transpose)
    solve_tt<T, FT, true>(sl, st);
  else
    solve_tt<T, FT, false>(sl, st);
}

void launch_band_solve(const SolveLaunch &sl, hipStream_t st) {
  if (sl.tile == 32) {
    if (sl.prec == 0) solve_t<32, double>(sl, st);
    else if (sl.prec == 1) solve_t<32, float>(sl, st);
    else solve_t<32, __hip_bfloat16>(sl, st);
  } else {
    if (sl.prec == 0) solve_t<16, double>(sl, st);
    else if (sl.prec == 1) solve_t<16, float>(sl, st);
    else solve_t<16, __hip_bfloat16>(sl, st);
  }
}

void launch_fill_int(int *y, int v, int N, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, y, v, N);
}
void launch_fill(double *y, double v, int64_t N, hipStream_t st) {
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((N + 255) / 256, 4096));
  hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(256), 0, st, y, v, N);
}

// ----------------------------------------------------------------------
// Fixed device scratch of the allocation-free entry points: one array per
// GPU, resident from the first load of this code object until the process
// ends.  Host code never passes the array's name to a kernel (on the host
// it is only a stand-in for the symbol): its device address is looked up
// once per device with hipGetSymbolAddress, with that device current, and
// that address is what kernels receive.
// ----------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

void *static_scratch() {
  static std::mutex mu;
  static std::vector<void *> addr;  // per device
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void *ptr = nullptr;
    HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(SEIRD_ERR_HIP, "no device address for the static scratch");
    addr[dev] = ptr;
  }
  return addr[dev];
}

void launch_gather_copies(const int64_t *gptr, const int32_t *gidx, const double *yloc, double *z, int add, int64_t N,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_gather_copies, dim3(nblocks(N)), dim3(256), 0, st, gptr, gidx, yloc, z, add, N);
}
void launch_coarse_restrict(const int64_t *zt_ptr, const int32_t *zt_col, const double *zt_val, const int32_t *cperm,
                            const double *r, double *rc, int64_t nc, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_restrict, dim3(nblocks(nc * 64)), dim3(256), 0, st, zt_ptr, zt_col, zt_val, cperm, r, rc,
                     nc);
}
void launch_coarse_prolong(const int64_t *z_ptr, const int32_t *z_col, const double *z_val, const int32_t *cperm,
                           const double *xc, double *z, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_prolong, dim3(nblocks(n)), dim3(256), 0, st, z_ptr, z_col, z_val, cperm, xc, z, n);
}

}  // namespace seird
