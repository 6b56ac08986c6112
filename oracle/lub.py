"""Near-field lubrication resistance, dense (oracle).

The paper adds a pairwise near-field resistance R_nf = R_2B - R_2B^inf
(Section 2.1) but never states its functions.  The model used here acts on
the *translational disturbance* velocity of bead pairs on different bodies
(Algorithm 1, step 1 restricts lubrication to inter-body pairs):

    R_pair = 6 pi eta a [ X(eps) n n + Y(eps) (I - n n) ],
    eps    = max(r/a - 2, eps_min),   n = (x_i - x_k) / r,
    X(eps) = 1/(4 eps) + (9/40) ln(1/eps) + (3/112) eps ln(1/eps) - 1/4,
    Y(eps) = (1/6) ln(1/eps),

the leading squeeze and shear terms of two equal spheres, shifted so that
both vanish at the cutoff r = 3a (eps = 1).  Rotational rows are zero.

What the pair resists is the relative velocity of the two bead centres with
the ambient rotation taken out, w = (u_i - u_k) - W d, d = x_i - x_k (the
minimum image), W the antisymmetric part of the velocity gradient; the force
on bead i is -sum_k R_pair w.  Its normal part is then the lab-frame rate at
which the gap closes, and a pair turning rigidly with the ambient vorticity
feels nothing.  Split into the two terms of Eq. `FH_agg`: with v = u - u_inf
the bead velocity relative to the ambient flow at its centre (Eq. `gc`),
w = (v_i - v_k) + E d, so the pair contributes -R_pair (v_i - v_k) to
-R_FU (U - U_inf) and -R_pair E d to R_FE : E_inf (`strain_forces`).  The sparse
preconditioner copy (Section 2.2.2: pairs with r < 2.1a) uses the same
functions with the smaller cutoff.

Surface roughness (Section 4.2, Eq. `tan_fric`) strengthens the tangential
(sliding) resistance below an asperity height h0: Y gains

    f(h) = alpha (a/h0) (h0/h - 3 h/h0 + 2 h^2/h0^2)  for h < h0, else 0,

with h = eps a the regularised gap.  The squeeze function X is unchanged, and
rolling is absent with the rotational rows; the FE and SE strengths belong to
the stresslet level.
"""
from __future__ import annotations

import math

import numpy as np


def X_squeeze(eps):
    eps = np.asarray(eps, dtype=float)
    lg = np.log(1.0 / eps)
    return 1.0 / (4.0 * eps) + 0.225 * lg + (3.0 / 112.0) * eps * lg - 0.25


def Y_shear(eps):
    return np.log(1.0 / np.asarray(eps, dtype=float)) / 6.0


def roughness(h, a, alpha, h0):
    """Tangential roughness correction f(h) (dimensionless, like Y)."""
    h = np.asarray(h, dtype=float)
    if alpha == 0:
        return np.zeros_like(h)
    t = h / h0
    return np.where(h < h0, alpha * (a / h0) * (1.0 / t - 3.0 * t + 2.0 * t * t), 0.0)


def min_image(d, L, strain=0.0):
    """Nearest image of separations d (..., 3) in the (sheared) lattice: y first, each
    period of y carrying gamma L of x, then x and z.  Exact for |d| < L/2."""
    d = np.array(d, dtype=float)
    ny = np.round(d[..., 1] / L)
    d[..., 1] -= ny * L
    d[..., 0] -= ny * strain * L
    d[..., 0] -= L * np.round(d[..., 0] / L)
    d[..., 2] -= L * np.round(d[..., 2] / L)
    return d


def pairs(x, body, L, r_cut, strain=0.0):
    """Inter-body bead pairs (i < k) with minimum-image distance < r_cut.

    Returns (i, k, d) with d = x_i - x_k (minimum image; strain as in `min_image`).
    Requires r_cut < L/2.
    """
    if r_cut <= 0:
        return np.zeros(0, int), np.zeros(0, int), np.zeros((0, 3))
    if r_cut >= L / 2:
        raise ValueError("lubrication cutoff must be below half the box side")
    n = len(x)
    d = min_image(x[:, None, :] - x[None, :, :], L, strain)
    r = np.linalg.norm(d, axis=-1)
    iu = np.triu_indices(n, 1)
    sel = (r[iu] < r_cut) & (body[iu[0]] != body[iu[1]])
    i, k = iu[0][sel], iu[1][sel]
    return i, k, d[i, k]


def pair_blocks(d, a, eta, eps_min=1e-3, rough=(0.0, 0.0)):
    """3x3 pair resistance blocks for separations d (m, 3); rough = (alpha, h0)."""
    r = np.linalg.norm(d, axis=1)
    n = d / r[:, None]
    eps = np.maximum(r / a - 2.0, eps_min)
    z = 6.0 * math.pi * eta * a
    X, Y = X_squeeze(eps), Y_shear(eps) + roughness(eps * a, a, *rough)
    nn = n[:, :, None] * n[:, None, :]
    return z * (X[:, None, None] * nn + Y[:, None, None] * (np.eye(3) - nn))


def strain_forces(x, body, L, a, eta, r_cut, E, eps_min=1e-3, rough=(0.0, 0.0), strain=0.0):
    """Bead forces (Nb, 3) of R_FE : E_inf at the bead level: -sum_k R_pair E d_ik over the
    inter-body pairs, d_ik = x_i - x_k (minimum image).  This is the near-field force on beads
    that all move with the ambient flow at their own centres."""
    n = len(x)
    f = np.zeros((n, 3))
    i, k, d = pairs(x, body, L, r_cut, strain)
    if len(i):
        B = pair_blocks(d, a, eta, eps_min, rough)
        g = np.einsum("mab,bc,mc->ma", B, np.asarray(E, dtype=float), d)
        np.add.at(f, i, -g)
        np.add.at(f, k, g)
    return f


def resistance_matrix(x, body, L, a, eta, r_cut, eps_min=1e-3, rough=(0.0, 0.0), strain=0.0):
    """Dense 6N x 6N R_nf (translational rows/columns only)."""
    n = len(x)
    R = np.zeros((n, 6, n, 6))
    i, k, d = pairs(x, body, L, r_cut, strain)
    if len(i):
        B = pair_blocks(d, a, eta, eps_min, rough)
        for m in range(len(i)):
            R[i[m], :3, i[m], :3] += B[m]
            R[k[m], :3, k[m], :3] += B[m]
            R[i[m], :3, k[m], :3] -= B[m]
            R[k[m], :3, i[m], :3] -= B[m]
    return R.reshape(6 * n, 6 * n)
