// Kernels of the 22-compartment model (Appendix C, Eqs. S ... D): residual,
// the per-compartment scalar systems of the decoupled sweep, stiffness.
// State layout [n][22], node-major, compartments in table order.
#include "kernels.h"

namespace seird {

namespace {

enum : int { S_ = 0, V_, E_, Q_, A_, W_, F_, B_, C_, X_, Y_, Z_, G_, N_, H_, H1_, I_, H2_, R1_, R2_, P_, D_ };

// compartment -> position in nu[] (-1: nodal)
__device__ inline int nu_slot(int c) {
  switch (c) {
    case S_: return 0;
    case V_: return 1;
    case E_: return 2;
    case A_: return 3;
    case F_: return 4;
    case B_: return 5;
    case C_: return 6;
    case P_: return 7;
    case R1_: return 8;
    case R2_: return 9;
    default: return -1;
  }
}

__device__ inline double nu_of(const seird22_params &p, int c) {
  const int k = nu_slot(c);
  return k < 0 ? 0.0 : p.nu[k];
}

// R_c(u) = s - d u_c with s, d free of u_c: inflow and loss rate of
// compartment c at one node (Appendix C, the right-hand side of its
// equation without the diffusion term)
__device__ inline void split22(int c, const double *u, const seird22_params &p, double &s, double &d) {
  const double lam = p.beta_A * u[A_] + p.beta_F * u[F_] + p.beta_B * u[B_] + p.beta_C * u[C_];
  const double rec = p.gamma_I * u[G_] + p.gamma_A * (u[F_] + u[X_]) + p.gamma_M * (u[B_] + u[Y_]);
  const double hosp = (1 - p.kappa_N) * p.gamma_S2 * u[N_] + (1 - p.kappa_H) * p.pi_H * u[H_] + p.pi_C * u[H2_];
  const double sev = p.gamma_S1 * (u[C_] + u[Z_]);
  const double vin = (1 - p.r_V) * lam * u[V_];  // infections among the vaccinated
  switch (c) {
    case S_: s = p.gamma_T * u[V_] + p.gamma_R * (u[R1_] + u[R2_]); d = lam + p.gamma_V; return;
    case V_: s = p.gamma_V * u[S_]; d = (1 - p.r_V) * lam + p.gamma_T; return;
    case E_: s = (1 - p.delta_S) * lam * u[S_] + (1 - p.delta_V) * vin; d = p.gamma_E; return;
    case Q_: s = p.delta_S * lam * u[S_] + p.delta_V * vin; d = p.gamma_E; return;
    case A_: s = p.gamma_E * u[E_]; d = p.gamma_P; return;
    case W_: s = p.gamma_E * u[Q_]; d = p.gamma_P; return;
    case F_: s = p.sigma_A * p.gamma_P * u[A_]; d = p.gamma_A + p.gamma_DA; return;
    case B_: s = (1 - p.sigma_A) * (1 - p.sigma_S) * p.gamma_P * u[A_]; d = p.gamma_M + p.gamma_DM; return;
    case C_: s = (1 - p.sigma_A) * p.sigma_S * p.gamma_P * u[A_]; d = p.gamma_S1; return;
    case X_: s = p.sigma_A * p.gamma_P * u[W_]; d = p.gamma_A + p.gamma_DA; return;
    case Y_: s = (1 - p.sigma_A) * (1 - p.sigma_S) * p.gamma_P * u[W_]; d = p.gamma_M + p.gamma_DM; return;
    case Z_: s = (1 - p.sigma_A) * p.sigma_S * p.gamma_P * u[W_]; d = p.gamma_S1; return;
    case G_: s = p.gamma_DA * (u[F_] + u[X_]) + p.gamma_DM * (u[B_] + u[Y_]); d = p.gamma_I; return;
    case N_: s = (1 - p.sigma_H) * sev; d = p.gamma_S2; return;
    case H_: s = p.sigma_H * (1 - p.sigma_C) * sev; d = p.pi_H; return;
    case H1_: s = p.sigma_H * p.sigma_C * sev; d = p.pi_A; return;
    case I_: s = p.pi_A * u[H1_]; d = p.pi_B; return;
    case H2_: s = (1 - p.kappa_I) * p.pi_B * u[I_]; d = p.pi_C; return;
    case R1_:
      s = (1 - p.phi_C) * ((1 - p.phi_M) * rec + (1 - p.phi_S) * hosp) + (1 - p.phi_P) * (1 - p.kappa_P) * p.gamma_C * u[P_];
      d = p.gamma_R;
      return;
    case R2_:
      s = (1 - p.phi_C) * (p.phi_M * rec + p.phi_S * hosp) + p.phi_P * (1 - p.kappa_P) * p.gamma_C * u[P_];
      d = p.gamma_R + p.gamma_L;
      return;
    case P_: s = p.phi_C * (rec + hosp); d = p.gamma_C; return;
    default:  // D
      s = p.kappa_H * p.pi_H * u[H_] + p.kappa_I * p.pi_B * u[I_] + p.kappa_N * p.gamma_S2 * u[N_] +
          p.gamma_L * u[R2_] + p.kappa_P * p.gamma_C * u[P_];
      d = 0.0;
      return;
  }
}

__device__ inline void load22(const double *__restrict__ src, double *dst) {
#pragma unroll
  for (int c = 0; c < SEIRD22_NC; ++c) dst[c] = src[c];
}

}  // namespace

// F = m (u - u^n) + dt nu_c K u_c - dt m R(u), one thread per node; the
// stiffness term gathers the node's elements (incidence records)
__global__ __launch_bounds__(256) void k22_residual(MeshDev m, seird22_params p, const double *__restrict__ u,
                                                    const double *__restrict__ up, double dt,
                                                    double *__restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  constexpr int NC22 = SEIRD22_NC;
  double ui[NC22];
  load22(u + NC22 * i, ui);
  constexpr int DIFF[10] = {S_, V_, E_, A_, F_, B_, C_, P_, R1_, R2_};
  double ku[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = m.inc_ptr[i]; k < m.inc_ptr[i + 1]; ++k) {
    const int64_t j = m.inc_j[k], l = m.inc_l[k];
    const double Kii = m.inc_K[3 * k], Kij = m.inc_K[3 * k + 1], Kil = m.inc_K[3 * k + 2];
#pragma unroll
    for (int q = 0; q < 10; ++q)
      ku[q] += Kii * ui[DIFF[q]] + Kij * u[NC22 * j + DIFF[q]] + Kil * u[NC22 * l + DIFF[q]];
  }
  const double mi = m.mass[i];
#pragma unroll
  for (int c = 0; c < NC22; ++c) {
    double s, d;
    split22(c, ui, p, s, d);
    const int q = nu_slot(c);
    const double diff = q < 0 ? 0.0 : dt * p.nu[q] * ku[q];
    F[NC22 * i + c] = mi * (ui[c] - up[NC22 * i + c]) + diff - dt * mi * (s - d * ui[c]);
  }
}

// plain P1 stiffness in node-graph form: Kd [n] (diagonal), Ko [slots]
__global__ __launch_bounds__(256) void k22_stiffness(MeshDev m, double *__restrict__ Kd, double *__restrict__ Ko) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m.n) {
    double a = 0.0;
    for (int64_t k = m.inc_ptr[t]; k < m.inc_ptr[t + 1]; ++k) a += m.inc_K[3 * k];
    Kd[t] = a;
  }
  if (t < m.nslots) {
    double o = 0.0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int32_t ek = m.slot_ek[2 * t + e];
      if (ek >= 0) o += m.inc_K[3 * (int64_t)(ek >> 1) + 1 + (ek & 1)];
    }
    Ko[t] = o;
  }
}

// compartment c's scalar system of the sweep, at the latest state u:
// diagonal m (1 + dt d_c) + dt nu_c Kd, right-hand side m u_c^n + dt m s_c.
// Nodal compartments (nu_c = 0) are solved in place (u_c = rhs / diag);
// diffusing ones get sdiag and the residual r = rhs - A u_c of the
// correction form (off-diagonal entries dt nu_c Ko).
__global__ __launch_bounds__(256) void k22_system(MeshDev m, seird22_params p, int c, double dt,
                                                  double *__restrict__ u, const double *__restrict__ up,
                                                  const double *__restrict__ Kd, const double *__restrict__ Ko,
                                                  double *__restrict__ sdiag, double *__restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  constexpr int NC22 = SEIRD22_NC;
  double ui[NC22];
  load22(u + NC22 * i, ui);
  double s, d;
  split22(c, ui, p, s, d);
  const double mi = m.mass[i];
  const double coef = dt * nu_of(p, c);
  const double diag = mi * (1.0 + dt * d) + coef * Kd[i];
  const double rhs = mi * up[NC22 * i + c] + dt * mi * s;
  if (coef == 0.0) {
    u[NC22 * i + c] = rhs / diag;
    return;
  }
  double au = diag * ui[c];
  for (int64_t t = m.rowptr[i]; t < m.rowptr[i + 1]; ++t) au += coef * Ko[t] * u[NC22 * (int64_t)m.col[t] + c];
  sdiag[i] = diag;
  r[i] = rhs - au;
}

__global__ __launch_bounds__(256) void k22_offdiag(int64_t ns, double coef, const double *__restrict__ Ko,
                                                   double *__restrict__ soff) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ns) soff[t] = coef * Ko[t];
}

__global__ __launch_bounds__(256) void k22_update(double *__restrict__ u, int c, const double *__restrict__ delta,
                                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) u[SEIRD22_NC * i + c] += delta[i];
}

// y = m ⊙ x per node (every compartment), for the residual's scale
__global__ __launch_bounds__(256) void k22_mass_scale(const double *__restrict__ mass, const double *__restrict__ x,
                                                      double *__restrict__ y, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < SEIRD22_NC * n) y[idx] = mass[idx / SEIRD22_NC] * x[idx];
}

// flags |= 1 for a nonfinite entry
__global__ __launch_bounds__(256) void k22_check(const double *__restrict__ u, int64_t N, int *flags) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < N && !isfinite(u[idx])) atomicOr(flags, 1);
}

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch22_residual(const MeshDev &m, const seird22_params &p, const double *u, const double *up, double dt,
                       double *F, hipStream_t st) {
  hipLaunchKernelGGL(k22_residual, dim3(nb256(m.n)), dim3(256), 0, st, m, p, u, up, dt, F);
}
void launch22_stiffness(const MeshDev &m, double *Kd, double *Ko, hipStream_t st) {
  hipLaunchKernelGGL(k22_stiffness, dim3(nb256(std::max(m.n, m.nslots))), dim3(256), 0, st, m, Kd, Ko);
}
void launch22_system(const MeshDev &m, const seird22_params &p, int c, double dt, double *u, const double *up,
                     const double *Kd, const double *Ko, double *sdiag, double *r, hipStream_t st) {
  hipLaunchKernelGGL(k22_system, dim3(nb256(m.n)), dim3(256), 0, st, m, p, c, dt, u, up, Kd, Ko, sdiag, r);
}
void launch22_offdiag(int64_t ns, double coef, const double *Ko, double *soff, hipStream_t st) {
  if (ns > 0) hipLaunchKernelGGL(k22_offdiag, dim3(nb256(ns)), dim3(256), 0, st, ns, coef, Ko, soff);
}
void launch22_update(double *u, int c, const double *delta, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k22_update, dim3(nb256(n)), dim3(256), 0, st, u, c, delta, n);
}
void launch22_mass_scale(const double *mass, const double *x, double *y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k22_mass_scale, dim3(nb256(SEIRD22_NC * n)), dim3(256), 0, st, mass, x, y, n);
}
void launch22_check(const double *u, int64_t N, int *flags, hipStream_t st) {
  hipLaunchKernelGGL(k22_check, dim3(nb256(N)), dim3(256), 0, st, u, N, flags);
}

}  // namespace seird
