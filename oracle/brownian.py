"""Brownian terms of the saddle system (oracle), Eq. `SP2` and Algorithm 1 step 3.

TEST INFRASTRUCTURE: used only by the tests, the smoke check and the CPU baseline.

With thermal energy kT and time step dt the right-hand side gains
  - the far-field slip velocity u_B = sqrt(2 kT / dt) (M_r^{1/2} psi_r + M_w^{1/2} psi_w)
    on the bead rows, with the PSE real/wave split of Section 2.2, and
  - the near-field force F_B = sqrt(2 kT / dt) R_nf^{1/2} psi_nf on the aggregate rows
    (through Sigma).
The method approximates the real-space and near-field square roots by Lanczos
iterations (Sections 2.2 and 2.5, after Chow and Saad); the oracle takes the exact symmetric
square roots by eigendecomposition of the dense matrices, so the Lanczos error is what
the comparison measures, or, where a fixed number of Lanczos steps is the point (the
lubrication matrix is singular, and the Lanczos root of a singular matrix converges
slowly), the k-step Lanczos approximation itself.
"""
from __future__ import annotations

import math

import numpy as np

from . import lub, pse


def sqrt_apply(A, z):
    """A^{1/2} z for a symmetric positive semi-definite A (eigenvalues below zero from
    rounding are clamped)."""
    A = np.asarray(A, dtype=float)
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    return V @ (np.sqrt(np.clip(w, 0.0, None)) * (V.T @ np.asarray(z, dtype=float)))


def lanczos_sqrt_apply(A, z, k):
    """The k-step Lanczos approximation |z| V_k T_k^{1/2} e_1 of A^{1/2} z (Chow and Saad):
    V_k an orthonormal basis of the Krylov space K_k(A, z) built from z / |z| by the
    three-term recurrence, each new vector orthogonalised against the whole basis (twice),
    and T_k = V_k^T A V_k the tridiagonal of the recurrence coefficients.  The basis stops
    early when the Krylov space is invariant (the new vector vanishes), and the result is
    then exact."""
    A = np.asarray(A, dtype=float)
    z = np.asarray(z, dtype=float)
    b0 = np.linalg.norm(z)
    if b0 == 0.0:
        return np.zeros_like(z)
    V = [z / b0]
    alpha, beta = [], []
    for j in range(k):
        w = A @ V[-1]
        scale = np.linalg.norm(w)
        B = np.array(V)
        w = w - B.T @ (B @ w)
        w = w - B.T @ (B @ w)
        alpha.append(float(V[-1] @ (A @ V[-1])))
        b = np.linalg.norm(w)
        if j + 1 == k or b <= 1e-14 * scale:
            break
        beta.append(b)
        V.append(w / b)
    T = np.diag(alpha) + np.diag(beta[:len(alpha) - 1], 1) + np.diag(beta[:len(alpha) - 1], -1)
    lam, Q = np.linalg.eigh(T)
    c = Q @ (np.sqrt(np.clip(lam, 0.0, None)) * Q[0])
    return b0 * (np.array(V[:len(alpha)]).T @ c)


def amplitude(kT, dt):
    return math.sqrt(2.0 * kT / dt)


def real_space_slip(x, L, a, eta, xi, r_cut, psi_r, kT, dt, strain=0.0):
    """sqrt(2 kT/dt) M_r^{1/2} psi_r (6 per bead) for the PSE real-space part."""
    Mr = pse.real_mobility(x, L, a, eta, xi, r_cut, strain)
    return amplitude(kT, dt) * sqrt_apply(Mr, np.ravel(psi_r)).reshape(-1, 6)


def near_field_force(x, body, L, a, eta, r_lub, psi_nf, kT, dt, eps_min=1e-3, rough=(0.0, 0.0), strain=0.0,
                     lanczos_steps=None):
    """sqrt(2 kT/dt) R_nf^{1/2} psi_nf: 3 per bead (the lubrication model acts on the
    translational rows only); rough = (alpha, h0) as in the lubrication model.  With
    lanczos_steps = k the root is the k-step Lanczos approximation instead of the exact one."""
    n = len(x)
    R = lub.resistance_matrix(x, body, L, a, eta, r_lub, eps_min, rough, strain).reshape(n, 6, n, 6)
    Rt = R[:, :3, :, :3].reshape(3 * n, 3 * n)
    z = np.ravel(psi_nf)
    root = sqrt_apply(Rt, z) if lanczos_steps is None else lanczos_sqrt_apply(Rt, z, lanczos_steps)
    return amplitude(kT, dt) * root.reshape(n, 3)
