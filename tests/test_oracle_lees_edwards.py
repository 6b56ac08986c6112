"""Pins of the oracle's sheared periodic lattice (Lees-Edwards), the boundary of long
steady-shear runs (Section 4.3).

Convention: at strain gamma the image of a point across the +y face sits gamma L further
along x, i.e. lattice vectors (L, 0, 0), (gamma L, L, 0), (0, 0, L); flow u_x = gamma_dot y
advances gamma by gamma_dot dt.

- the convention itself: a bead just below the +y face meets the image of a bead just above
  the -y face at the offset gamma L, and folding y moves x by -gamma L;
- the nearest image equals brute force over explicit lattice vectors;
- strains gamma and gamma + 1 give the same lattice, hence the same mobility;
- the Ewald sum on the sheared lattice does not depend on the splitting parameter;
- mirroring x maps strain gamma to -gamma (velocities as vectors, angular velocities as
  pseudovectors).
"""
import itertools

import numpy as np

from oracle import forces, lub, pse, rigid, rpy

L = 7.0


def test_image_convention():
    g = 0.3
    x0 = np.array([0.4, L / 2 - 0.2, 0.1])
    x1 = x0 + np.array([0.0, 2.1, 0.0]) - np.array([g * L, L, 0.0])  # its image across +y is x0 + 2.1 e_y
    i, k, d = lub.pairs(np.array([x0, x1]), np.array([0, 1]), L, 3.0, strain=g)
    assert len(i) == 1 and np.allclose(d[0], [0.0, -2.1, 0.0], atol=1e-12)
    assert len(lub.pairs(np.array([x0, x1]), np.array([0, 1]), L, 3.0, strain=-g)[0]) == 0
    w = rigid.wrap(np.array([[0.2, L / 2 + 0.3, 0.0]]), L, strain=g)
    assert np.allclose(w, [[0.2 - g * L, -L / 2 + 0.3, 0.0]])


def test_nearest_image_is_brute_force():
    rng = np.random.default_rng(1)
    n = np.array(list(itertools.product(range(-3, 4), repeat=3)), dtype=float)
    for g in (0.0, 0.37, -0.5, 0.49):
        A = n.copy()
        A[:, 0] += g * A[:, 1]
        for d in rng.uniform(-1.6 * L, 1.6 * L, size=(200, 3)):
            best = d + L * A[np.argmin(np.linalg.norm(d + L * A, axis=1))]
            got = lub.min_image(d, L, g)
            if np.linalg.norm(best) < 0.45 * L:  # within reach of every cutoff used (< L/2)
                assert np.allclose(got, best, atol=1e-12)


def _beads():
    rng = np.random.default_rng(2)
    return rng.uniform(-L / 2, L / 2, size=(4, 3))


def test_strain_period_one():
    x = _beads()
    for g in (0.3, -0.45):
        M0 = rpy.periodic_mobility(x, L, xi=0.9, strain=g)
        M1 = rpy.periodic_mobility(x, L, xi=0.9, strain=g + 1.0)
        assert np.abs(M1 - M0).max() <= 1e-12 * np.abs(M0).max()
    Mc = rpy.periodic_mobility(x, L, xi=0.9)
    assert np.abs(rpy.periodic_mobility(x, L, xi=0.9, strain=1.0) - Mc).max() <= 1e-12 * np.abs(Mc).max()
    assert np.abs(rpy.periodic_mobility(x, L, xi=0.9, strain=0.3) - Mc).max() > 1e-4 * np.abs(Mc).max()


def test_ewald_split_independent_on_sheared_lattice():
    x = _beads()
    Ma = rpy.periodic_mobility(x, L, xi=0.7, strain=0.41)
    Mb = rpy.periodic_mobility(x, L, xi=1.3, strain=0.41)
    assert np.abs(Ma - Mb).max() <= 1e-11 * np.abs(Ma).max()


def test_mirror_maps_strain_to_minus_strain():
    x = _beads()
    P = np.diag([-1.0, 1.0, 1.0])
    T = np.zeros((6, 6))
    T[:3, :3], T[3:, 3:] = P, -P  # angular velocity and torque are pseudovectors
    Tn = np.kron(np.eye(len(x)), T)
    M = rpy.periodic_mobility(x, L, xi=0.9, strain=0.33)
    Mm = rpy.periodic_mobility(x @ P, L, xi=0.9, strain=-0.33)
    assert np.abs(M - Tn @ Mm @ Tn).max() <= 1e-12 * np.abs(M).max()


def test_force_images_agree_with_nearest_image_pairs():
    rng = np.random.default_rng(3)
    x = rng.uniform(-L / 2, L / 2, size=(30, 3))
    body = np.arange(30)
    g = -0.38
    f = forces.bead_forces(x, body, L, 1.0, 2.6, strain=g, Z=1.0, kappa=1.0)
    i, k, d = lub.pairs(x, body, L, 2.6, strain=g)
    assert len(i) > 3
    ref = np.zeros_like(f)
    for a, b, dv in zip(i, k, d):
        r = np.linalg.norm(dv)
        fv = forces.pair_force(np.array([r]), 1.0, Z=1.0, kappa=1.0)[0] * dv / r
        ref[a] += fv
        ref[b] -= fv
    assert np.allclose(f, ref, atol=1e-12)


def test_pse_split_sums_to_the_ewald_mobility_on_sheared_lattice():
    """The PSE (Hasimoto) real- and wave-space parts on the sheared lattice add up to the
    Beenakker-split mobility on the same lattice: two different splits of one lattice sum."""
    x = _beads()[:3]
    g, xi = -0.31, 0.8
    Mr = pse.real_mobility(x, L, 1.0, 1.0, xi, 7.0 / xi, strain=g)
    Mw = pse.wave_mobility(x, L, 1.0, 1.0, xi, strain=g)
    M = rpy.periodic_mobility(x, L, xi=0.9, strain=g)
    assert np.abs(Mr + Mw - M).max() <= 1e-9 * np.abs(M).max()
