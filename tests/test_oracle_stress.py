"""Pins of the oracle's constraint stresslet (Section 3.1.4, Eq. `stress_comp`).

- A rigid doublet of touching beads held along the axis of a uniaxial extension: the two
  beads would separate at the relative velocity 2 a e' (rate e'), the rod holds them, and
  by the free-space RPY mobility at contact (self 1/(6 pi eta a), pair along the line of
  centres 5/(48 pi eta a)) each bead feels 16 pi eta a^2 e' outwards, so S_xx =
  32 pi eta a^3 e' and every other component vanishes (periodic images change it by
  O((a/L)^3)).
- Covariance under the cubic rotations of the periodic box, and linearity in the flow.
- A planted sign error in the hydrodynamic force fails the doublet pin.
"""
import math

import numpy as np
import pytest

import fsdgen
from oracle import rigid, saddle, stress

A, ETA = 1.0, 1.0


def _doublet_stresslet(L, rate=1.0):
    xb = np.array([[1.0, 0, 0], [-1.0, 0, 0]])
    G = rate * np.diag([1.0, -0.5, -0.5])
    U, F, _, asm = saddle.solve(L, A, ETA, [0, 2], xb, np.zeros((1, 3)), np.array([[1.0, 0, 0, 0]]),
                                np.zeros((1, 6)), G)
    return stress.constraint_stresslets(asm, F, U - asm.Uinf, [0, 2], L, A, ETA, 0.0, G)[0]


def test_doublet_in_extension_matches_rpy_contact_value():
    ref = 32.0 * math.pi * ETA * A ** 3
    S = _doublet_stresslet(80.0)
    assert abs(S[0, 0] - ref) < 2e-3 * ref
    off = S.copy()
    off[0, 0] = 0.0
    assert np.abs(off).max() < 1e-10 * ref
    # the periodic correction shrinks with the box as (a/L)^3
    d40, d80 = abs(_doublet_stresslet(40.0)[0, 0] - ref), abs(S[0, 0] - ref)
    assert 4.0 < d40 / d80 < 12.0


def test_doublet_pin_catches_a_flipped_force(monkeypatch):
    real = stress.constraint_stresslets

    def flipped(asm, F, *a, **k):
        return real(asm, -np.asarray(F), *a, **k)
    monkeypatch.setattr(stress, "constraint_stresslets", flipped)
    S = _doublet_stresslet(80.0)
    assert abs(S[0, 0] - 32.0 * math.pi) > 1.0


def _cluster_case(seed=3):
    rng = fsdgen.rng_from(seed)
    shapes = [fsdgen.sticking_cluster(rng, nb) for nb in (4, 3, 5)]
    L = 12.0
    com, quat = fsdgen.place_clusters(rng, shapes, L, gap=0.1)
    offs = np.r_[0, np.cumsum([len(s) for s in shapes])].astype(np.int32)
    return L, offs, np.concatenate(shapes), com, quat


def _stresslets(L, offs, xb, com, quat, G):
    U, F, _, asm = saddle.solve(L, A, ETA, offs, xb, com, quat, np.zeros((len(offs) - 1, 6)), G, r_lub=3.0)
    return stress.constraint_stresslets(asm, F, U - asm.Uinf, offs, L, A, ETA, 3.0, G)


def test_stresslets_covariant_under_cubic_rotation_and_linear_in_flow():
    L, offs, xb, com, quat = _cluster_case()
    G = np.zeros((3, 3))
    G[0, 1] = 1.0
    S = _stresslets(L, offs, xb, com, quat, G)
    R = np.array([[0.0, -1, 0], [1, 0, 0], [0, 0, 1]])  # a quarter turn about z: a symmetry of the cube
    qR = np.array([math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4)])

    def qmul(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b
        return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    quat2 = np.array([qmul(qR, q) for q in quat])
    S2 = _stresslets(L, offs, xb, com @ R.T, quat2, R @ G @ R.T)
    assert np.allclose(S2, R @ S @ R.T, atol=1e-10 * np.abs(S).max())
    assert np.allclose(_stresslets(L, offs, xb, com, quat, 2.5 * G), 2.5 * S, atol=1e-10 * np.abs(S).max())
