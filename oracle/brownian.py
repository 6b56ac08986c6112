"""Brownian terms of the saddle system (oracle), Eq. `SP2` and Algorithm 1 step 3.

TEST INFRASTRUCTURE: used only by the tests, the smoke check and the CPU baseline.

With thermal energy kT and time step dt the right-hand side gains
  - the far-field slip velocity u_B = sqrt(2 kT / dt) (M_r^{1/2} psi_r + M_w^{1/2} psi_w)
    on the bead rows, with the PSE real/wave split of Section 2.2, and
  - the near-field force F_B = sqrt(2 kT / dt) R_nf^{1/2} psi_nf on the aggregate rows
    (through Sigma).
The method approximates the real-space and near-field square roots by Lanczos
iterations; the oracle takes the exact symmetric square roots by eigendecomposition
of the dense matrices, so the Lanczos error is what the comparison measures.
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


def amplitude(kT, dt):
    return math.sqrt(2.0 * kT / dt)


def real_space_slip(x, L, a, eta, xi, r_cut, psi_r, kT, dt, strain=0.0):
    """sqrt(2 kT/dt) M_r^{1/2} psi_r (6 per bead) for the PSE real-space part."""
    Mr = pse.real_mobility(x, L, a, eta, xi, r_cut, strain)
    return amplitude(kT, dt) * sqrt_apply(Mr, np.ravel(psi_r)).reshape(-1, 6)


def near_field_force(x, body, L, a, eta, r_lub, psi_nf, kT, dt, eps_min=1e-3, rough=(0.0, 0.0), strain=0.0):
    """sqrt(2 kT/dt) R_nf^{1/2} psi_nf: 3 per bead (the lubrication model acts on the
    translational rows only); rough = (alpha, h0) as in the lubrication model."""
    n = len(x)
    R = lub.resistance_matrix(x, body, L, a, eta, r_lub, eps_min, rough, strain).reshape(n, 6, n, 6)
    Rt = R[:, :3, :, :3].reshape(3 * n, 3 * n)
    return amplitude(kT, dt) * sqrt_apply(Rt, np.ravel(psi_nf)).reshape(n, 3)
