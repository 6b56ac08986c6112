"""Constraint stresslet of rigid aggregates (oracle), Section 3.1.4, Eq. `stress_comp`.

TEST INFRASTRUCTURE: used only by the tests.

At the force-torque level each bead carries no stresslet of its own, so the particle
stress of an aggregate comes from the non-uniform distribution of force over its beads:
the constraint stress S^C_j = -(1/2) sum_i [(x_i - X_j) F^C_i + ((x_i - X_j) F^C_i)^T],
with F^C_i minus the sum of all forces on bead i.  Here those forces are the far-field
hydrodynamic force F_i (the force moments of Eq. `spm_agg`: by Eq. `mob_rel` the fluid's
force on the beads, M F = -(u - u_inf)), the near-field lubrication force and the
bead-level conservative force, so

    S^C_j = sum_{i in j} sym(r_i (F_i + f_nf,i + f_P,i)),   r_i = x_i - X_j,

and the suspension's particle stress is (1/V) sum_j S^C_j.  The near-field force on
bead i is what lubrication exerts at the solved velocities (reading of `lub`):
-sum_k R_pair [(u_i - u_k) - W d_ik] with u the lab-frame bead velocities.
"""
from __future__ import annotations

import numpy as np

from . import lub, rigid


def near_field_forces(A, V, offsets, L, a, eta, r_lub, grad_u, eps_min=1e-3, rough=(0.0, 0.0), strain=0.0):
    """Lubrication force on each bead (Nb, 3) at the aggregate velocities V (N, 6) relative to
    the imposed flow, for the assembled system A (see saddle.assemble)."""
    nb = len(A.x)
    body = rigid.body_index(offsets)
    v = (A.Sig.T @ np.asarray(V, dtype=float).reshape(-1)).reshape(nb, 6)
    E, _ = rigid.strain_and_spin(grad_u)
    # velocity relative to the imposed flow at the bead centre (Eq. `gc`)
    v[:, :3] -= A.r @ E.T
    f = -(A.Rnf @ v.reshape(-1)).reshape(nb, 6)[:, :3]
    if r_lub > 0:
        f += lub.strain_forces(A.x, body, L, a, eta, r_lub, E, eps_min, rough, strain)
    return f


def constraint_stresslets(A, F, V, offsets, L, a, eta, r_lub, grad_u, f_pair=None, **kw):
    """S^C per aggregate (N, 3, 3) from the bead force moments F (Nb, 6) and the aggregate
    velocities V relative to the imposed flow (N, 6); f_pair: bead conservative forces."""
    offsets = np.asarray(offsets)
    body = rigid.body_index(offsets)
    f = np.asarray(F, dtype=float).reshape(-1, 6)[:, :3].copy()
    f = f + near_field_forces(A, V, offsets, L, a, eta, r_lub, grad_u, **kw)
    if f_pair is not None:
        f = f + np.asarray(f_pair, dtype=float).reshape(-1, 3)
    outer = A.r[:, :, None] * f[:, None, :]
    S = np.zeros((len(offsets) - 1, 3, 3))
    np.add.at(S, body, 0.5 * (outer + outer.transpose(0, 2, 1)))
    return S
