"""Explicit Euler update of rigid aggregates (oracle), Section 2.4.

Eq. `EM1`: X <- X + U dt.
Eq. `EM2`: q <- q + (dt/2) (0, W) (x) q, then normalise; the printed
"W x q" is read as the quaternion product of the pure quaternion (0, W)
with q.
Eq. `EM3`: x_i = X_j + R(q_j) x_body,i (bead positions rebuilt from the
body frame; the printed x(t) on the right-hand side is read as X).
Centroids are wrapped into [-L/2, L/2)^3 after each step.
"""
from __future__ import annotations

import numpy as np

from . import rigid


def quat_mul(p, q):
    """Hamilton product of quaternions (..., 4) in (w, x, y, z) order."""
    pw, pv = p[..., :1], p[..., 1:]
    qw, qv = q[..., :1], q[..., 1:]
    w = pw * qw - np.sum(pv * qv, axis=-1, keepdims=True)
    v = pw * qv + qw * pv + np.cross(pv, qv)
    return np.concatenate([w, v], axis=-1)


def euler_step(com, quat, U, dt, L, strain=0.0):
    """One step; centroids folded into the lattice of the given (end-of-step) strain."""
    U = np.asarray(U, dtype=float).reshape(-1, 6)
    X = np.asarray(com, dtype=float) + U[:, :3] * dt
    om = np.concatenate([np.zeros((len(U), 1)), U[:, 3:]], axis=1)
    q = np.asarray(quat, dtype=float)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    q = q + 0.5 * dt * quat_mul(om, q)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    return rigid.wrap(X, L, strain), q
