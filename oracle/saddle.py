"""Aggregate saddle-point system, assembled densely and solved directly (oracle).

Eq. `spm_agg` (Section 2.3.3) at force-torque level (no stresslet rows):

    [ M      Sigma^T ] [ F_h ]   [ b1 ]
    [ Sigma  -R_agg  ] [  V  ] = [ b2 ],     R_agg = Sigma R_nf Sigma^T,

F_h = hydrodynamic (force, torque) on the beads, V = U - U_inf per aggregate
(translation, rotation), and

    b1_i = (E_inf r_i + u_B,i, w_B,i),
    b2_j = -(F_P,j + [Sigma F_B,nf]_j + [R_FE : E_inf]_j),

The right-hand side uses E_inf (x - X) as printed in Eq. `spm_agg` (derived
from Eq. `gc`); the table of Section 2.3.3 prints the opposite sign.

The aggregate term R_FE : E_inf of Eq. `FH_agg` is the near-field force on
the aggregates when each moves with the ambient flow at its centroid
(V = 0).  By Eq. `gc` the beads then move relative to the ambient flow at
their own centres by -e_i, e_i = (E_inf r_i, 0); the bead-level pair force
adds -R_pair E d_ik (see `lub`), so

    R_FE : E_inf = Sigma (R_nf e + f_E),   f_E,i = -sum_k R_pair E_inf d_ik,

which makes every inter-body pair resist the lab-frame closing of its gap.

The block-triangular preconditioner (Section 2.3.3 and its table; Algorithm 1
step 1) approximates M by the bead self-mobility M~ = diag(mu_t I, mu_r I) and
the Schur complement by -blockdiag_j[Sigma (M~^-1 + R~_nf) Sigma^T]_jj with
R~_nf the lubrication restricted to r < 2.1a:

    P^-1 = [[I, -M~^-1 Sigma^T], [0, I]] [[M~^-1, 0], [0, S~^-1]] [[I, 0], [-Sigma M~^-1, I]].
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np
import scipy.linalg as sla

from . import lub, rigid, rpy


@dataclass
class Assembled:
    M: np.ndarray            # 6Nb x 6Nb mobility
    Rnf: np.ndarray          # 6Nb x 6Nb lubrication
    Sig: np.ndarray          # 6N x 6Nb
    Ragg: np.ndarray         # 6N x 6N
    b1: np.ndarray
    b2: np.ndarray
    Uinf: np.ndarray         # (N, 6) ambient (translation, rotation) at each centroid
    x: np.ndarray            # bead positions (Nb, 3)
    r: np.ndarray            # body vectors (Nb, 3)
    com: np.ndarray          # wrapped centroids (N, 3)


def assemble(L, a, eta, offsets, x_body, com, quat, force, grad_u, r_lub=0.0,
             eps_min=1e-3, xi=None, u_brown=None, f_brown_nf=None, M=None, rough=(0.0, 0.0), strain=0.0):
    offsets = np.asarray(offsets)
    nb, na = int(offsets[-1]), len(offsets) - 1
    xb = rigid.centre_bodies(x_body, offsets)
    X = rigid.wrap(np.asarray(com, dtype=float), L, strain)
    r = rigid.bead_vectors(quat, xb, offsets)
    body = rigid.body_index(offsets)
    x = X[body] + r
    if M is None:
        M = rpy.periodic_mobility(x, L, a, eta, xi=xi, strain=strain)
    Rnf = lub.resistance_matrix(x, body, L, a, eta, r_lub, eps_min, rough, strain)
    Sig = rigid.sigma_matrix(r, offsets)
    Ragg = Sig @ Rnf @ Sig.T
    E, W = rigid.strain_and_spin(grad_u)
    e = np.zeros((nb, 6))
    e[:, :3] = r @ E.T
    b1 = e.copy()
    if u_brown is not None:
        b1 += np.asarray(u_brown).reshape(nb, 6)
    fb = np.asarray(force, dtype=float).reshape(na * 6).copy()
    if f_brown_nf is not None:
        fb += Sig @ np.asarray(f_brown_nf).reshape(nb * 6)
    fe = Rnf @ e.reshape(-1)
    if r_lub > 0:
        fE = lub.strain_forces(x, body, L, a, eta, r_lub, E, eps_min, rough, strain)
        fe.reshape(nb, 6)[:, :3] += fE
    b2 = -(fb + Sig @ fe)
    G = np.asarray(grad_u, dtype=float)
    Uinf = np.zeros((na, 6))
    Uinf[:, :3] = X @ G.T
    Uinf[:, 3:] = W
    return Assembled(M, Rnf, Sig, Ragg, b1.reshape(-1), b2, Uinf, x, r, X)


def saddle_matrix(A: Assembled):
    return np.block([[A.M, A.Sig.T], [A.Sig, -A.Ragg]])


def rhs(A: Assembled):
    return np.concatenate([A.b1, A.b2])


def solve_schur(A: Assembled):
    """V = (Sigma M^-1 Sigma^T + R_agg)^-1 (Sigma M^-1 b1 - b2); F = M^-1 (b1 - Sigma^T V)."""
    c = sla.cho_factor(A.M, lower=True)
    MiSt = sla.cho_solve(c, A.Sig.T)
    Mib1 = sla.cho_solve(c, A.b1)
    S = A.Sig @ MiSt + A.Ragg
    V = np.linalg.solve(S, A.Sig @ Mib1 - A.b2)
    F = sla.cho_solve(c, A.b1 - A.Sig.T @ V)
    return F, V


def solve_lu(A: Assembled):
    K = saddle_matrix(A)
    y = sla.solve(K, rhs(A))
    n1 = A.M.shape[0]
    return y[:n1], y[n1:]


def residual(A: Assembled, F, V):
    K = saddle_matrix(A)
    b = rhs(A)
    return float(np.linalg.norm(b - K @ np.concatenate([F, V])) / np.linalg.norm(b))


def preconditioner(A: Assembled, offsets, a, eta, L, r_pre=2.1, eps_min=1e-3):
    """Dense P^-1 of the block-triangular factorisation (see module docstring)."""
    offsets = np.asarray(offsets)
    nb, na = int(offsets[-1]), len(offsets) - 1
    body = rigid.body_index(offsets)
    Rt = lub.resistance_matrix(A.x, body, L, a, eta, r_pre * a if r_pre > 0 else 0.0, eps_min)
    drag = np.tile(np.r_[np.full(3, 6 * math.pi * eta * a), np.full(3, 8 * math.pi * eta * a ** 3)], nb)
    Minv = np.diag(drag)
    # keep only the bead-diagonal 6x6 blocks of R~ (inter-body couplings dropped)
    Rt_d = np.zeros_like(Rt)
    for i in range(nb):
        s = slice(6 * i, 6 * i + 6)
        Rt_d[s, s] = Rt[s, s]
    Sfull = A.Sig @ (Minv + Rt_d) @ A.Sig.T
    Sblk = np.zeros_like(Sfull)
    for j in range(na):
        s = slice(6 * j, 6 * j + 6)
        Sblk[s, s] = np.linalg.inv(Sfull[s, s])
    Sinv = -Sblk
    n1 = 6 * nb
    I1, I2 = np.eye(n1), np.eye(6 * na)
    Z12, Z21 = np.zeros((n1, 6 * na)), np.zeros((6 * na, n1))
    L3 = np.block([[I1, Z12], [-A.Sig @ Minv, I2]])
    D = np.block([[Minv, Z12], [Z21, Sinv]])
    U3 = np.block([[I1, -Minv @ A.Sig.T], [Z21, I2]])
    return U3 @ D @ L3


def gmres(K, b, Pinv=None, tol=1e-10, restart=50, maxit=2000):
    """Right-preconditioned restarted GMRES with modified Gram-Schmidt (textbook).

    Returns (x, iterations, relative residual).
    """
    n = len(b)
    if Pinv is None:
        Pinv = np.eye(n)
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    its = 0
    while its < maxit:
        r = b - K @ x
        beta = np.linalg.norm(r)
        if beta / bn <= tol:
            break
        Q = np.zeros((n, restart + 1))
        H = np.zeros((restart + 1, restart))
        Q[:, 0] = r / beta
        g = np.zeros(restart + 1)
        g[0] = beta
        cs, sn = np.zeros(restart), np.zeros(restart)
        k_used = 0
        for k in range(restart):
            w = K @ (Pinv @ Q[:, k])
            for j in range(k + 1):
                H[j, k] = Q[:, j] @ w
                w -= H[j, k] * Q[:, j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                Q[:, k + 1] = w / H[k + 1, k]
            for j in range(k):
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            k_used = k + 1
            if abs(g[k + 1]) / bn <= tol or its >= maxit:
                break
        y = sla.solve_triangular(H[:k_used, :k_used], g[:k_used])
        x = x + Pinv @ (Q[:, :k_used] @ y)
    r = b - K @ x
    return x, its, float(np.linalg.norm(r) / bn)


def solve(L, a, eta, offsets, x_body, com, quat, force, grad_u, r_lub=0.0, eps_min=1e-3,
          xi=None, u_brown=None, f_brown_nf=None, rough=(0.0, 0.0), strain=0.0):
    """Aggregate velocities U (N, 6) = V + U_inf, bead forces F (Nb, 6), residual;
    rough = (alpha, h0) adds the tangential roughness correction to lubrication; strain is
    that of a sheared periodic lattice."""
    A = assemble(L, a, eta, offsets, x_body, com, quat, force, grad_u, r_lub, eps_min, xi,
                 u_brown, f_brown_nf, rough=rough, strain=strain)
    F, V = solve_schur(A)
    na = len(offsets) - 1
    U = V.reshape(na, 6) + A.Uinf
    return U, F.reshape(-1, 6), residual(A, F, V), A


def solve_suspension(s, **kw):
    """Convenience wrapper taking a workload object with the usual attributes."""
    return solve(s.L, s.a, s.eta, s.offsets, s.x_body, s.com, s.quat, s.force, s.grad_u,
                 r_lub=s.r_lub, **kw)
