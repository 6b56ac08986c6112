"""Conservative bead-pair forces (oracle), Section 4.2 and Eq. `dlvo_potential`.

TEST INFRASTRUCTURE: used only by the tests, the smoke check and the CPU baseline.

Between beads of radius a that belong to different bodies, at centre distance r
(separation h = r - 2a):

- van der Waals: the Hamaker sphere-sphere potential for equal radii,
      V(s) = -(A/6) [2a^2/(s^2 - 4a^2) + 2a^2/s^2 + ln((s^2 - 4a^2)/s^2)],
  evaluated at s = r + h_c (the separation regularised by h_c); for overlapping beads
  (h < 0) the force keeps its value at contact;
- double layer: V(r) = (a^2 / r) Z exp(-kappa (r - 2a));
- Hertz contact: f = k_n delta^1.5 along the line of centres, delta = 2a - r > 0.

The forces of the two potentials are -dV/dr along the unit vector from the other bead.
Reading: the first term of the printed potential carries a_2 squared, which would leave
the bracket with a dimension; the standard sphere-sphere form with 2 a_1 a_2 is used.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def vdw_potential(r, a, hamaker, h_c):
    """V_vdW at centre distance r (r + h_c > 2a)."""
    s = np.asarray(r, dtype=float) + h_c
    s2, c = s * s, 4.0 * a * a
    return -(hamaker / 6.0) * (2 * a * a / (s2 - c) + 2 * a * a / s2 + np.log((s2 - c) / s2))


def double_layer_potential(r, a, Z, kappa):
    r = np.asarray(r, dtype=float)
    return (a * a / r) * Z * np.exp(-kappa * (r - 2 * a))


def vdw_force(r, a, hamaker, h_c):
    """-dV/dr of the van der Waals potential (positive = repulsive), held at contact."""
    s = np.maximum(np.asarray(r, dtype=float), 2 * a) + h_c
    s2, c = s * s, 4.0 * a * a
    dV = -(hamaker / 6.0) * (-4 * a * a * s / (s2 - c) ** 2 - 4 * a * a / s ** 3 + 2 * s / (s2 - c) - 2 / s)
    return -dV


def double_layer_force(r, a, Z, kappa):
    r = np.asarray(r, dtype=float)
    return Z * a * a * np.exp(-kappa * (r - 2 * a)) * (1 / (r * r) + kappa / r)


def hertz_force(r, a, k_n):
    d = np.maximum(2 * a - np.asarray(r, dtype=float), 0.0)
    return k_n * d ** 1.5


def pair_force(r, a, k_n=0.0, hamaker=0.0, Z=0.0, kappa=0.0, h_c=0.0):
    """Signed magnitude along the unit vector from the other bead."""
    f = np.zeros_like(np.asarray(r, dtype=float))
    if hamaker:
        f = f + vdw_force(r, a, hamaker, h_c)
    if Z:
        f = f + double_layer_force(r, a, Z, kappa)
    if k_n:
        f = f + hertz_force(r, a, k_n)
    return f


def bead_forces(x, body, L, a, r_cut, strain=0.0, **coef):
    """Force on every bead (n, 3): brute force over bead pairs of different bodies and over
    periodic images within r_cut (image n at (n_x + gamma n_y, n_y, n_z) L for strain gamma)."""
    x = np.asarray(x, dtype=float)
    n = len(x)
    m = int(math.ceil(r_cut / L)) + 1
    shifts = np.array(list(itertools.product(range(-m, m + 1), repeat=3)), dtype=float)
    shifts[:, 0] += strain * shifts[:, 1]
    shifts *= L
    f = np.zeros((n, 3))
    for i in range(n):
        for j in range(n):
            if body[i] == body[j]:
                continue
            d = x[i] - x[j] + shifts  # every image of j
            r = np.linalg.norm(d, axis=1)
            near = (r < r_cut) & (r > 0)
            if not near.any():
                continue
            g = pair_force(r[near], a, **coef) / r[near]
            f[i] += (g[:, None] * d[near]).sum(axis=0)
    return f
