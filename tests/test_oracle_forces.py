"""Pins of the conservative-force oracle (Section 4.2) to facts other than its own formulas:
derivatives of the potentials by finite differences, the far-field and near-contact limits
of the Hamaker sphere-sphere potential, the Hertz contact energy, and the symmetries of the
pair sum (Newton's third law, translation invariance, periodic images)."""
import numpy as np
import pytest

from oracle import forces

A, Z, KAPPA, HC, KN = 1.3, 2.0, 1.7, 0.02, 50.0
a = 1.0


@pytest.mark.parametrize("r", [2.05, 2.3, 3.0, 4.5])
def test_forces_are_minus_the_potential_gradient(r):
    h = 1e-6
    dv = (forces.vdw_potential(r + h, a, A, HC) - forces.vdw_potential(r - h, a, A, HC)) / (2 * h)
    assert forces.vdw_force(r, a, A, HC) == pytest.approx(-dv, rel=1e-7)
    dd = (forces.double_layer_potential(r + h, a, Z, KAPPA) - forces.double_layer_potential(r - h, a, Z, KAPPA)) / (2 * h)
    assert forces.double_layer_force(r, a, Z, KAPPA) == pytest.approx(-dd, rel=1e-7)


def test_vdw_far_field_is_the_r6_law():
    # two spheres far apart: V -> -(16/9) A a^6 / s^6 (1 + O(a^2/s^2)); the bracket's terms
    # cancel to O(a^6/s^6), so the check stays where rounding is far below that correction
    for s, rel in ((60.0, 2e-3), (100.0, 1e-3)):
        v = forces.vdw_potential(s - HC, a, A, HC)
        assert v * s ** 6 == pytest.approx(-16.0 / 9.0 * A * a ** 6, rel=rel)


def test_vdw_near_contact_is_the_derjaguin_limit():
    # equal spheres at small gap g: V -> -A a / (12 g) (effective radius a/2)
    g = 1e-5
    v = forces.vdw_potential(2 * a + g - HC, a, A, HC)
    assert v * g == pytest.approx(-A * a / 12.0, rel=1e-3)


def test_vdw_force_held_at_contact_for_overlaps():
    fc = forces.vdw_force(2 * a, a, A, HC)
    assert fc < 0  # attractive
    for r in (1.9, 1.99, 1.5):
        assert forces.vdw_force(r, a, A, HC) == fc


def test_hertz_force_integrates_to_the_contact_energy():
    # work against the contact force from r to contact: (2/5) k_n delta^(5/2)
    from scipy.integrate import quad
    for d in (0.01, 0.1, 0.3):
        w, _ = quad(lambda r: forces.hertz_force(r, a, KN), 2 * a - d, 2 * a, epsabs=1e-14, epsrel=1e-12)
        assert w == pytest.approx(0.4 * KN * d ** 2.5, rel=1e-9)
    assert forces.hertz_force(2 * a, a, KN) == 0 and forces.hertz_force(2.5, a, KN) == 0


def _config(rng, n_body=6, per=3, L=9.0):
    x = rng.uniform(-L / 2, L / 2, size=(n_body * per, 3))
    body = np.repeat(np.arange(n_body), per)
    return x, body, L


def test_pair_sum_obeys_newtons_third_law_and_translation():
    rng = np.random.default_rng(3)
    x, body, L = _config(rng)
    coef = dict(k_n=KN, hamaker=A, Z=Z, kappa=KAPPA, h_c=HC)
    f = forces.bead_forces(x, body, L, a, 3.0, **coef)
    assert np.abs(f.sum(axis=0)).max() < 1e-10 * np.abs(f).max()
    shift = np.array([0.7, -1.1, 2.3])
    xs = (x + shift + L / 2) % L - L / 2
    assert np.allclose(forces.bead_forces(xs, body, L, a, 3.0, **coef), f, rtol=1e-12, atol=1e-12)


def test_pair_across_the_boundary_equals_the_unwrapped_pair():
    L, coef = 10.0, dict(k_n=KN, hamaker=A, Z=Z, kappa=KAPPA, h_c=HC)
    x = np.array([[4.6, 0.2, -0.1], [-4.7, 0.1, 0.3]])  # 0.7 apart through the x face... plus images
    f = forces.bead_forces(x, np.array([0, 1]), L, a, 3.0, **coef)
    d = x[0] - (x[1] + np.array([L, 0, 0]))
    r = np.linalg.norm(d)
    want = forces.pair_force(r, a, **coef) / r * d
    assert np.allclose(f[0], want, rtol=1e-13) and np.allclose(f[1], -want, rtol=1e-13)
