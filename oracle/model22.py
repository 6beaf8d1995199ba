"""The 22-compartment SEIRD model of Appendix C on P1 triangles (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Compartments, in the order of the compartment table of Appendix C (index in
brackets): S[0] V[1] E[2] Q[3] A[4] W[5] F[6] B[7] C[8] X[9] Y[10] Z[11]
G[12] N[13] H[14] H1[15] I[16] H2[17] R1[18] R2[19] P[20] D[21].  Ten of them
diffuse with constant coefficients (S, V, E, A, F, B, C, P, R1, R2); the
rest are nodal ODEs.  The reaction terms are the right-hand sides of the
Appendix C equations (Eqs. S ... D), written out term by term below.

Readings where the paper is silent (each also listed with the design notes):

* the force of infection lambda is not defined in Appendix C; it is taken as
  mass action in the densities of the four infectious compartments that
  move and do not isolate, lambda = beta_A A + beta_F F + beta_B B + beta_C C,
  the same density-dependent form as the S I and S E terms of the
  five-compartment model (Eqs. seird1-5);
* the parameter table names phi_A ("acute COVID") while the equations use
  phi_C for the same split; phi_C is used;
* no values are given: the inputs module supplies synthetic rates of a
  plausible magnitude (per day), used only to exercise the discretisation;
* space and time as for the five-compartment model: lumped mass, backward
  Euler, homogeneous Neumann data, so the discrete system is
  F_c(u) = m (u_c - u_c^n) + dt nu_c K u_c - dt m R_c(u) = 0, K the P1
  stiffness matrix;
* the solver is the decoupled Picard-Gauss-Seidel iteration of Appendix A
  applied compartment by compartment in table order: each R_c is affine in
  u_c given the others, R_c = s_c - d_c u_c, and every sweep solves
  (m (1 + dt d_c) + dt nu_c K) u_c = m u_c^n + dt m s_c with the latest
  values of the other compartments, until
  ||u^{k+1} - u^k|| / ||u^n|| <= tol (the test of Eq. picardtol).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Geometry

NAMES = ["S", "V", "E", "Q", "A", "W", "F", "B", "C", "X", "Y", "Z", "G", "N", "H", "H1", "I", "H2",
         "R1", "R2", "P", "D"]
NC22 = len(NAMES)
IX = {nm: k for k, nm in enumerate(NAMES)}
DIFFUSING = ["S", "V", "E", "A", "F", "B", "C", "P", "R1", "R2"]


def nu_all(p) -> np.ndarray:
    """Diffusion coefficient of every compartment (0 for the nodal ones);
    ``p.nu`` lists those of S V E A F B C P R1 R2 in that order."""
    v = np.zeros(NC22)
    for nm, x in zip(DIFFUSING, p.nu):
        v[IX[nm]] = x
    return v


def _cols(u):
    return {nm: u[..., k] for k, nm in enumerate(NAMES)}


def force_of_infection(u, p):
    c = _cols(u)
    return p.beta_A * c["A"] + p.beta_F * c["F"] + p.beta_B * c["B"] + p.beta_C * c["C"]


def reaction22(u: np.ndarray, p) -> np.ndarray:
    """R(u) [..., 22]: the right-hand sides of Eqs. S ... D of Appendix C
    (without the diffusion terms)."""
    c = _cols(u)
    lam = force_of_infection(u, p)
    S, V, E, Q, A, W = c["S"], c["V"], c["E"], c["Q"], c["A"], c["W"]
    F, B, C, X, Y, Z = c["F"], c["B"], c["C"], c["X"], c["Y"], c["Z"]
    G, N, H, H1, I, H2 = c["G"], c["N"], c["H"], c["H1"], c["I"], c["H2"]
    R1, R2, P = c["R1"], c["R2"], c["P"]
    # recoveries from the infectious and the hospital tracks
    phi = p.gamma_I * G + p.gamma_A * (F + X) + p.gamma_M * (B + Y)
    psi = (1 - p.kappa_N) * p.gamma_S2 * N + (1 - p.kappa_H) * p.pi_H * H + p.pi_C * H2
    sev = p.gamma_S1 * (C + Z)
    R = np.empty(u.shape)
    R[..., IX["S"]] = -lam * S - p.gamma_V * S + p.gamma_T * V + p.gamma_R * (R1 + R2)
    R[..., IX["V"]] = -(1 - p.r_V) * lam * V + p.gamma_V * S - p.gamma_T * V
    R[..., IX["E"]] = (1 - p.delta_S) * lam * S + (1 - p.delta_V) * (1 - p.r_V) * lam * V - p.gamma_E * E
    R[..., IX["Q"]] = p.delta_S * lam * S + p.delta_V * (1 - p.r_V) * lam * V - p.gamma_E * Q
    R[..., IX["A"]] = p.gamma_E * E - p.gamma_P * A
    R[..., IX["W"]] = p.gamma_E * Q - p.gamma_P * W
    R[..., IX["F"]] = p.sigma_A * p.gamma_P * A - p.gamma_A * F - p.gamma_DA * F
    R[..., IX["B"]] = (1 - p.sigma_A) * (1 - p.sigma_S) * p.gamma_P * A - p.gamma_M * B - p.gamma_DM * B
    R[..., IX["C"]] = (1 - p.sigma_A) * p.sigma_S * p.gamma_P * A - p.gamma_S1 * C
    R[..., IX["X"]] = p.sigma_A * p.gamma_P * W - p.gamma_A * X - p.gamma_DA * X
    R[..., IX["Y"]] = (1 - p.sigma_A) * (1 - p.sigma_S) * p.gamma_P * W - p.gamma_M * Y - p.gamma_DM * Y
    R[..., IX["Z"]] = (1 - p.sigma_A) * p.sigma_S * p.gamma_P * W - p.gamma_S1 * Z
    R[..., IX["G"]] = p.gamma_DA * (F + X) + p.gamma_DM * (B + Y) - p.gamma_I * G
    R[..., IX["N"]] = (1 - p.sigma_H) * sev - p.gamma_S2 * N
    R[..., IX["H"]] = p.sigma_H * (1 - p.sigma_C) * sev - p.pi_H * H
    R[..., IX["H1"]] = p.sigma_H * p.sigma_C * sev - p.pi_A * H1
    R[..., IX["I"]] = p.pi_A * H1 - p.pi_B * I
    R[..., IX["H2"]] = (1 - p.kappa_I) * p.pi_B * I - p.pi_C * H2
    R[..., IX["R1"]] = ((1 - p.phi_C) * ((1 - p.phi_M) * phi + (1 - p.phi_S) * psi)
                        + (1 - p.phi_P) * (1 - p.kappa_P) * p.gamma_C * P - p.gamma_R * R1)
    R[..., IX["R2"]] = ((1 - p.phi_C) * (p.phi_M * phi + p.phi_S * psi)
                        + p.phi_P * (1 - p.kappa_P) * p.gamma_C * P - p.gamma_R * R2 - p.gamma_L * R2)
    R[..., IX["P"]] = p.phi_C * (phi + psi) - p.gamma_C * P
    R[..., IX["D"]] = (p.kappa_H * p.pi_H * H + p.kappa_I * p.pi_B * I + p.kappa_N * p.gamma_S2 * N
                       + p.gamma_L * R2 + p.kappa_P * p.gamma_C * P)
    return R


def split22(k: int, u: np.ndarray, p):
    """(s_k, d_k) with R_k(u) = s_k - d_k u_k, s_k and d_k free of u_k (the
    affine dependence of compartment k's reaction on its own density)."""
    c = _cols(u)
    nm = NAMES[k]
    lam = force_of_infection(u, p)
    phi = p.gamma_I * c["G"] + p.gamma_A * (c["F"] + c["X"]) + p.gamma_M * (c["B"] + c["Y"])
    psi = (1 - p.kappa_N) * p.gamma_S2 * c["N"] + (1 - p.kappa_H) * p.pi_H * c["H"] + p.pi_C * c["H2"]
    sev = p.gamma_S1 * (c["C"] + c["Z"])
    z = np.zeros_like(c["S"])
    if nm == "S":
        return p.gamma_T * c["V"] + p.gamma_R * (c["R1"] + c["R2"]), lam + p.gamma_V
    if nm == "V":
        return p.gamma_V * c["S"], (1 - p.r_V) * lam + p.gamma_T
    if nm == "E":
        return (1 - p.delta_S) * lam * c["S"] + (1 - p.delta_V) * (1 - p.r_V) * lam * c["V"], z + p.gamma_E
    if nm == "Q":
        return p.delta_S * lam * c["S"] + p.delta_V * (1 - p.r_V) * lam * c["V"], z + p.gamma_E
    if nm == "A":
        # (lambda enters only the S, V, E and Q equations)
        return p.gamma_E * c["E"], z + p.gamma_P
    if nm == "W":
        return p.gamma_E * c["Q"], z + p.gamma_P
    if nm == "F":
        return p.sigma_A * p.gamma_P * c["A"], z + p.gamma_A + p.gamma_DA
    if nm == "B":
        return (1 - p.sigma_A) * (1 - p.sigma_S) * p.gamma_P * c["A"], z + p.gamma_M + p.gamma_DM
    if nm == "C":
        return (1 - p.sigma_A) * p.sigma_S * p.gamma_P * c["A"], z + p.gamma_S1
    if nm == "X":
        return p.sigma_A * p.gamma_P * c["W"], z + p.gamma_A + p.gamma_DA
    if nm == "Y":
        return (1 - p.sigma_A) * (1 - p.sigma_S) * p.gamma_P * c["W"], z + p.gamma_M + p.gamma_DM
    if nm == "Z":
        return (1 - p.sigma_A) * p.sigma_S * p.gamma_P * c["W"], z + p.gamma_S1
    if nm == "G":
        return p.gamma_DA * (c["F"] + c["X"]) + p.gamma_DM * (c["B"] + c["Y"]), z + p.gamma_I
    if nm == "N":
        return (1 - p.sigma_H) * sev, z + p.gamma_S2
    if nm == "H":
        return p.sigma_H * (1 - p.sigma_C) * sev, z + p.pi_H
    if nm == "H1":
        return p.sigma_H * p.sigma_C * sev, z + p.pi_A
    if nm == "I":
        return p.pi_A * c["H1"], z + p.pi_B
    if nm == "H2":
        return (1 - p.kappa_I) * p.pi_B * c["I"], z + p.pi_C
    if nm == "R1":
        return ((1 - p.phi_C) * ((1 - p.phi_M) * phi + (1 - p.phi_S) * psi)
                + (1 - p.phi_P) * (1 - p.kappa_P) * p.gamma_C * c["P"]), z + p.gamma_R
    if nm == "R2":
        return ((1 - p.phi_C) * (p.phi_M * phi + p.phi_S * psi)
                + p.phi_P * (1 - p.kappa_P) * p.gamma_C * c["P"]), z + p.gamma_R + p.gamma_L
    if nm == "P":
        return p.phi_C * (phi + psi), z + p.gamma_C
    if nm == "D":
        return (p.kappa_H * p.pi_H * c["H"] + p.kappa_I * p.pi_B * c["I"] + p.kappa_N * p.gamma_S2 * c["N"]
                + p.gamma_L * c["R2"] + p.kappa_P * p.gamma_C * c["P"]), z
    raise ValueError(nm)


def stiffness(geo: Geometry) -> sp.csr_matrix:
    """P1 stiffness K_ij = int grad phi_i . grad phi_j (sum of K^T)."""
    tri = geo.tri
    r = np.repeat(tri, 3, axis=1).ravel()
    c = np.tile(tri, (1, 3)).ravel()
    return sp.coo_matrix((geo.K.ravel(), (r, c)), shape=(geo.n, geo.n)).tocsr()


def residual22(u, u_prev, dt, geo: Geometry, p, K=None) -> np.ndarray:
    """F(u) [n, 22] = m (u - u^n) + dt nu K u - dt m R(u)."""
    K = stiffness(geo) if K is None else K
    m = geo.mass[:, None]
    return m * (u - u_prev) + dt * (K @ u) * nu_all(p)[None, :] - dt * m * reaction22(u, p)


def picard_gs_step22(u_prev, dt, geo: Geometry, p, tol=1e-10, max_sweeps=100, K=None):
    """One backward-Euler step by compartment-wise Picard-Gauss-Seidel
    sweeps; returns (u, eps_hist)."""
    K = stiffness(geo) if K is None else K
    m = geo.mass
    nu = nu_all(p)
    u = u_prev.copy()
    unorm = np.linalg.norm(u_prev)
    hist = []
    for _ in range(max_sweeps):
        uk = u.copy()
        for k in range(NC22):
            s, d = split22(k, u, p)
            rhs = m * u_prev[:, k] + dt * m * s
            diag = m * (1.0 + dt * d)
            if nu[k] != 0.0:
                A = (sp.diags(diag) + dt * nu[k] * K).tocsc()
                u[:, k] = spla.spsolve(A, rhs)
            else:
                u[:, k] = rhs / diag
        eps = np.linalg.norm(u - uk) / unorm
        hist.append(eps)
        if eps <= tol:
            return u, hist
    raise RuntimeError(f"Picard-Gauss-Seidel did not converge: {hist[-3:]}")
