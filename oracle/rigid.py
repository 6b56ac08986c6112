"""Rigid-body kinematics of bead aggregates (oracle).

Geometric constraint (Section 2.3.1, Eqs. `gc` and `sigma`): for bead i of
aggregate j, with body vector r_i = x_i - X_j,

    Sigma_{j,i} = [[I, 0], [[r_i]x, I]],

so Sigma maps bead (force, torque) to aggregate (sum f, sum (t + r x f)) and
Sigma^T maps aggregate (U, W) to bead (U + W x r_i, W).  The Levi-Civita
block of Eq. `sigma` is read as r x (.) acting on forces.

Bead positions follow Eq. `EM3` read as x_i = X_j + R(q_j) x_body,i, where
R(q) is the rotation of the unit quaternion q = (w, x, y, z).
"""
from __future__ import annotations

import numpy as np


def rotation_matrix(q):
    """Rotation matrices of unit quaternions (..., 4) in (w, x, y, z) order."""
    q = np.asarray(q, dtype=float)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def body_index(offsets):
    offsets = np.asarray(offsets)
    return np.repeat(np.arange(len(offsets) - 1), np.diff(offsets))


def centre_bodies(x_body, offsets):
    """Shift each aggregate's body vectors to zero mean (centroid = COM)."""
    xb = np.array(x_body, dtype=float)
    for j in range(len(offsets) - 1):
        s = slice(offsets[j], offsets[j + 1])
        xb[s] -= xb[s].mean(axis=0)
    return xb


def bead_vectors(quat, x_body, offsets):
    """Lab-frame body vectors r_i = R(q_j) x_body,i."""
    b = body_index(offsets)
    R = rotation_matrix(quat)
    return np.einsum("iab,ib->ia", R[b], x_body)


def wrap(X, L, strain=0.0):
    """Fold points into the primary cell [-L/2, L/2)^3.  With a sheared lattice (strain
    gamma: the image across the +y face sits at +gamma L in x), y is folded first and every
    crossing moves x by -gamma L per period before x and z are folded."""
    X = np.array(X, dtype=float)
    if strain:
        ny = np.floor((X[..., 1] + L / 2) / L)
        X[..., 1] -= ny * L
        X[..., 0] -= ny * strain * L
    return (X + L / 2) % L - L / 2


def sigma_matrix(r, offsets):
    """Dense Sigma (6N x 6Ntot)."""
    nb, na = len(r), len(offsets) - 1
    b = body_index(offsets)
    S = np.zeros((na, 6, nb, 6))
    for i in range(nb):
        j = b[i]
        S[j, :3, i, :3] = np.eye(3)
        S[j, 3:, i, 3:] = np.eye(3)
        rx, ry, rz = r[i]
        S[j, 3:, i, :3] = [[0, -rz, ry], [rz, 0, -rx], [-ry, rx, 0]]
    return S.reshape(6 * na, 6 * nb)


def strain_and_spin(grad_u):
    """E_inf = sym(grad u), W_inf = (1/2) curl u for grad_u[a, b] = d u_a / d x_b."""
    G = np.asarray(grad_u, dtype=float)
    E = 0.5 * (G + G.T)
    W = 0.5 * np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
    return E, W
