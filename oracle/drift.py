"""Brownian drift (oracle), Appendix A: random finite differences (Eq. `rfd`) and
Fixman's midpoint scheme.

TEST INFRASTRUCTURE: used only by the tests, the smoke check and the CPU baseline.

The drift kT div N of the aggregate mobility N = R_FU^{-1} is estimated from one Gaussian
vector dq (6 per aggregate: translation, rotation) by two saddle solves at the displaced
configurations q +- (eps/2) dq, each with right-hand side (0, -dq) (a force and torque dq on
every aggregate, no ambient flow and no other forcing):

    U_drift = kT (U+ - U-) / eps.

Readings: a displacement of the generalised coordinates moves each centroid by (eps/2) dq_t
and turns each body by the exact rotation with rotation vector (eps/2) dq_r (quaternion
(cos(phi/2), sin(phi/2) phi_hat) applied on the left); eps defaults to gmres_tol^(1/3) a.
"""
from __future__ import annotations

import numpy as np

from . import integrate, rigid, saddle


def rotate(quat, phi):
    """Quaternions turned by the rotation vectors phi (N, 3): q <- r(phi) (x) q."""
    phi = np.asarray(phi, dtype=float).reshape(-1, 3)
    ang = np.linalg.norm(phi, axis=1)
    axis = np.where(ang[:, None] > 0, phi / np.where(ang > 0, ang, 1.0)[:, None], 0.0)
    r = np.concatenate([np.cos(ang / 2)[:, None], np.sin(ang / 2)[:, None] * axis], axis=1)
    q = integrate.quat_mul(r, np.asarray(quat, dtype=float))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def displace(com, quat, dq, h, L, strain=0.0):
    dq = np.asarray(dq, dtype=float).reshape(-1, 6)
    X = rigid.wrap(np.asarray(com, dtype=float) + h * dq[:, :3], L, strain)
    return X, rotate(quat, h * dq[:, 3:])


def mobility_velocity(L, a, eta, offsets, x_body, com, quat, ft, r_lub=0.0, xi=None, strain=0.0):
    """U = N(q) ft: the saddle solve with aggregate forces and torques ft and nothing else
    (on the lattice of the given strain)."""
    na = len(offsets) - 1
    U, *_ = saddle.solve(L, a, eta, offsets, x_body, com, quat, np.asarray(ft, dtype=float).reshape(na, 6),
                         np.zeros((3, 3)), r_lub=r_lub, xi=xi, strain=strain)
    return U


def rfd_drift(L, a, eta, offsets, x_body, com, quat, dq, eps, kT, r_lub=0.0, xi=None, strain=0.0):
    """kT (U+ - U-) / eps for the given Gaussian vector dq (N, 6)."""
    Xp, qp = displace(com, quat, dq, +0.5 * eps, L, strain)
    Xm, qm = displace(com, quat, dq, -0.5 * eps, L, strain)
    Up = mobility_velocity(L, a, eta, offsets, x_body, Xp, qp, dq, r_lub, xi, strain)
    Um = mobility_velocity(L, a, eta, offsets, x_body, Xm, qm, dq, r_lub, xi, strain)
    return kT * (Up - Um) / eps


def mobility_matrix(L, a, eta, offsets, x_body, com, quat, r_lub=0.0, xi=None):
    """Dense aggregate mobility N (6N x 6N), column by column."""
    na = len(offsets) - 1
    cols = []
    for k in range(6 * na):
        e = np.zeros(6 * na)
        e[k] = 1.0
        cols.append(mobility_velocity(L, a, eta, offsets, x_body, com, quat, e, r_lub, xi).ravel())
    return np.array(cols).T


def divergence(L, a, eta, offsets, x_body, com, quat, h=1e-4, r_lub=0.0, xi=None):
    """kT-free divergence (div N)_i = sum_k dN_ik / dq_k by central differences of the dense
    mobility along every generalised coordinate (brute force, tiny systems only)."""
    na = len(offsets) - 1
    div = np.zeros(6 * na)
    for k in range(6 * na):
        e = np.zeros(6 * na)
        e[k] = 1.0
        Xp, qp = displace(com, quat, e, +h, L)
        Xm, qm = displace(com, quat, e, -h, L)
        Np = mobility_matrix(L, a, eta, offsets, x_body, Xp, qp, r_lub, xi)
        Nm = mobility_matrix(L, a, eta, offsets, x_body, Xm, qm, r_lub, xi)
        div += (Np[:, k] - Nm[:, k]) / (2 * h)
    return div.reshape(na, 6)


def brownian_velocity(L, a, eta, offsets, x_body, com, quat, u_b, f_b, r_lub=0.0, xi=None, strain=0.0):
    """Aggregate velocities of the saddle solve whose right-hand side holds only the given
    Brownian slip u_b (6 per bead) and near-field force f_b (3 per bead)."""
    na = len(offsets) - 1
    fb6 = np.zeros((len(f_b), 6))
    fb6[:, :3] = np.asarray(f_b, dtype=float).reshape(-1, 3)
    U, *_ = saddle.solve(L, a, eta, offsets, x_body, com, quat, np.zeros((na, 6)), np.zeros((3, 3)), r_lub=r_lub,
                         xi=xi, u_brown=np.asarray(u_b, dtype=float).reshape(-1, 6), f_brown_nf=fb6, strain=strain)
    return U


def fixman_drift(L, a, eta, offsets, x_body, com, quat, u_b, f_b, m, dt, r_lub=0.0, xi=None, strain=0.0):
    """Fixman's midpoint estimate (Appendix A): U0 from the Brownian terms at x, the
    configuration advanced by U0 dt/m (on the same lattice), U' from the same Brownian terms
    there, and drift = (m/2) (U' - U0)."""
    U0 = brownian_velocity(L, a, eta, offsets, x_body, com, quat, u_b, f_b, r_lub, xi, strain)
    X1, q1 = integrate.euler_step(com, quat, U0, dt / m, L, strain)
    U1 = brownian_velocity(L, a, eta, offsets, x_body, X1, q1, u_b, f_b, r_lub, xi, strain)
    return 0.5 * m * (U1 - U0)
