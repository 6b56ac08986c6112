"""Pins of the oracle's roughness correction to the tangential lubrication resistance
(Section 4.2, Eq. `tan_fric`).

f(h) = alpha (a/h0) (c1 h0/h + c2 h/h0 + c3 h^2/h0^2) on h < h0 is fixed by three facts of the
model, each checked here without its formula: the resistance diverges as alpha a / h at
contact (c1 = 1), it switches on continuously at h0 (c1 + c2 + c3 = 0) and with zero slope
(-c1 + c2 + 2 c3 = 0).  Those give c = (1, -3, 2); the curvature at h0 then follows
(f ~ 3 alpha a delta^2 / h0^3 at h = h0 - delta).  The pair blocks carry the correction on the
sliding directions only, as a relative-motion resistance.
"""
import math

import numpy as np

from oracle import lub, rigid

a, eta = 1.0, 1.0
alpha, h0 = 0.7, 0.08


def test_divergence_at_contact():
    for h in (1e-7, 1e-8):
        assert abs(h * lub.roughness(h, a, alpha, h0) / (alpha * a) - 1.0) < 1e-5


def test_switches_on_smoothly_at_the_asperity_height():
    assert lub.roughness(h0, a, alpha, h0) == 0.0
    assert np.all(lub.roughness(np.array([h0 * 1.0001, 2 * h0, 0.5]), a, alpha, h0) == 0.0)
    for d in (1e-3 * h0, 1e-4 * h0):
        f = float(lub.roughness(h0 - d, a, alpha, h0))
        assert abs(f / d) < 4 * alpha * a * d / h0 ** 3          # zero slope at h0
        assert abs(f / d ** 2 / (3 * alpha * a / h0 ** 3) - 1) < 5 * d / h0  # the curvature that follows
    h = np.linspace(0.01, 0.999, 50) * h0
    assert np.all(lub.roughness(h, a, alpha, h0) > 0)           # strengthens, never weakens


def _pair(gap, direction, rad=a):
    n = np.asarray(direction, dtype=float)
    n /= np.linalg.norm(n)
    x = np.array([np.zeros(3), (2 * rad + gap) * n])
    return x, np.array([0, 1]), n


def test_pair_blocks_sliding_only():
    rad, H0 = 1.7, 1.7 * h0  # a radius other than 1 tells gaps from reduced gaps
    z = 6 * math.pi * eta * rad
    for gap in (0.5 * H0, 0.9 * H0, 1.5 * H0):
        x, body, n = _pair(gap, [0.3, -0.5, 0.8], rad)
        R0 = lub.resistance_matrix(x, body, 20.0, rad, eta, 3.0 * rad)
        R1 = lub.resistance_matrix(x, body, 20.0, rad, eta, 3.0 * rad, rough=(alpha, H0))
        t = np.cross(n, [1.0, 0, 0])
        t /= np.linalg.norm(t)
        f = alpha * (rad / gap) * (1 - gap / H0) ** 2 * (1 + 2 * gap / H0) if gap < H0 else 0.0
        for v_rel, extra in ((t, z * f), (n, 0.0)):
            v = np.zeros((2, 6))
            v[0, :3] = v_rel  # bead 0 moves, bead 1 at rest
            F0, F1 = (R0 @ v.ravel()).reshape(2, 6), (R1 @ v.ravel()).reshape(2, 6)
            assert np.allclose(F1[0, :3] - F0[0, :3], extra * v_rel, atol=1e-12 * z)
            assert np.allclose(F1[1, :3] - F0[1, :3], -extra * v_rel, atol=1e-12 * z)
        u = np.zeros((2, 6))
        u[:, :3] = [0.2, 0.4, -0.1]  # common translation: no relative motion, no force
        assert np.abs(R1 @ u.ravel()).max() < 1e-10 * z
        assert np.linalg.eigvalsh(R1).min() > -1e-9 * z


def test_same_body_pairs_untouched():
    x, _, _ = _pair(0.3 * h0, [0, 0, 1])
    R = lub.resistance_matrix(x, np.array([0, 0]), 20.0, a, eta, 3.0, rough=(alpha, h0))
    assert np.abs(R).max() == 0
    assert rigid.body_index(np.array([0, 2])).tolist() == [0, 0]
