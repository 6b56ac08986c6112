"""Pins of the random-finite-difference drift oracle (Appendix A, Eq. `rfd`).

- The estimator averaged over Gaussian dq is the divergence of the aggregate mobility N,
  because E[dq dq^T] = I.  The same identity holds exactly for the basis vectors: the sum of
  the estimator over dq = e_k equals the divergence sum_k dN_ik/dq_k computed from dense
  mobility matrices at displaced configurations (a different path through the oracle).
- One sphere in a periodic box has a mobility independent of its position and orientation,
  so every estimate is zero.
- The rotations are the exact ones: they agree with scipy's rotation-vector rotations.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import drift, rigid

L, a, eta = 8.0, 1.0, 1.0


def _two_bodies():
    offs = np.array([0, 2, 3], dtype=np.int32)
    xb = np.array([[-1.05, 0, 0], [1.05, 0, 0], [0, 0, 0]])
    com = np.array([[0.0, 0, 0], [0.3, 2.6, 0.4]])
    quat = np.array([[1.0, 0, 0, 0], [0.9, 0.1, 0.2, 0.3]])
    return offs, xb, com, quat / np.linalg.norm(quat, axis=1, keepdims=True)


def test_rotations_are_exact():
    rng = np.random.default_rng(5)
    q = rng.normal(size=(4, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    phi = rng.normal(size=(4, 3)) * 0.7
    q2 = drift.rotate(q, phi)
    for k in range(4):
        want = Rotation.from_rotvec(phi[k]).as_matrix() @ rigid.rotation_matrix(q[k])
        assert np.allclose(rigid.rotation_matrix(q2[k]), want, atol=1e-13)
    assert np.allclose(drift.rotate(q2, -phi), q, atol=1e-13)


def test_estimator_over_the_basis_sums_to_the_divergence():
    offs, xb, com, quat = _two_bodies()
    div = drift.divergence(L, a, eta, offs, xb, com, quat, h=1e-4)
    eps = 2e-4
    est = np.zeros_like(div)
    for k in range(12):
        e = np.zeros(12)
        e[k] = 1.0
        est += drift.rfd_drift(L, a, eta, offs, xb, com, quat, e.reshape(2, 6), eps, kT=1.0)
    assert np.abs(div).max() > 1e-4  # a configuration with drift
    assert np.abs(est - div).max() <= 1e-6 * np.abs(div).max() + 1e-12


def test_single_sphere_has_no_drift():
    offs = np.array([0, 1], dtype=np.int32)
    dq = np.random.default_rng(6).normal(size=(1, 6))
    d = drift.rfd_drift(L, a, eta, offs, np.zeros((1, 3)), np.array([[0.4, -1.0, 2.0]]),
                        np.array([[1.0, 0, 0, 0]]), dq, 1e-2, kT=1.0)
    assert np.abs(d).max() < 1e-9


def _brownian_terms(rng, nb):
    return rng.normal(size=(nb, 6)), rng.normal(size=(nb, 3))


def test_fixman_single_sphere_has_no_drift():
    offs = np.array([0, 1], dtype=np.int32)
    ub, fb = _brownian_terms(np.random.default_rng(8), 1)
    d = drift.fixman_drift(L, a, eta, offs, np.zeros((1, 3)), np.array([[0.4, -1.0, 2.0]]),
                           np.array([[1.0, 0, 0, 0]]), ub, fb, m=100, dt=1e-3)
    assert np.abs(d).max() < 1e-9


def test_fixman_large_m_is_the_directional_derivative():
    """(m/2)(U' - U0) -> (dt/2) (dN/dq . U0) f for large m, when the Brownian terms act as a
    fixed generalised force f (U0 = N f): two spheres, near-field force only.  The derivative
    comes from central differences of the aggregate mobility along U0 (the displacement path
    of the random finite differences)."""
    offs = np.array([0, 1, 2], dtype=np.int32)
    xb = np.zeros((2, 3))
    com = np.array([[0.0, 0.2, 0.0], [2.4, -0.3, 0.5]])
    quat = np.tile([1.0, 0, 0, 0], (2, 1))
    fb = np.random.default_rng(9).normal(size=(2, 3))
    ub = np.zeros((2, 6))
    dt, m = 1e-2, 1e4
    est = drift.fixman_drift(L, a, eta, offs, xb, com, quat, ub, fb, m, dt)
    U0 = drift.brownian_velocity(L, a, eta, offs, xb, com, quat, ub, fb)
    f = np.zeros((2, 6))
    f[:, :3] = fb  # the near-field force acts like an external force on each sphere
    assert np.allclose(drift.mobility_matrix(L, a, eta, offs, xb, com, quat) @ f.ravel(), U0.ravel(), atol=1e-12)
    h = 1e-4
    Xp, qp = drift.displace(com, quat, U0, +h, L)
    Xm, qm = drift.displace(com, quat, U0, -h, L)
    dN = (drift.mobility_matrix(L, a, eta, offs, xb, Xp, qp) - drift.mobility_matrix(L, a, eta, offs, xb, Xm, qm)) / (2 * h)
    want = (0.5 * dt * dN @ f.ravel()).reshape(-1, 6)
    assert np.abs(want).max() > 1e-8
    assert np.abs(est - want).max() <= 1e-3 * np.abs(want).max()
