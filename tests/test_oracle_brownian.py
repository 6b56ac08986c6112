"""Pins of the oracle's Brownian terms (Eq. `SP2`, Algorithm 1 step 3)."""
import math

import numpy as np

import fsdgen
from oracle import brownian, lub, pse, rigid


def test_sqrt_apply_squares_back_and_matches_diagonal():
    rng = np.random.default_rng(3)
    B = rng.normal(size=(12, 12))
    A = B @ B.T + 0.1 * np.eye(12)
    S = np.column_stack([brownian.sqrt_apply(A, e) for e in np.eye(12)])
    assert np.allclose(S, S.T, atol=1e-12)
    assert np.allclose(S @ S, A, rtol=0, atol=1e-11 * np.abs(A).max())
    d = rng.uniform(0.5, 4.0, 7)
    z = rng.normal(size=7)
    assert np.allclose(brownian.sqrt_apply(np.diag(d), z), np.sqrt(d) * z, atol=1e-14)


def test_fluctuation_dissipation_amplitude():
    """<u u^T> = (2 kT / dt) M for u = sqrt(2 kT/dt) M^{1/2} psi, psi standard normal."""
    rng = np.random.default_rng(4)
    B = rng.normal(size=(6, 6))
    M = B @ B.T + np.eye(6)
    kT, dt = 0.7, 0.01
    K = 200000
    psi = rng.normal(size=(6, K))
    w, V = np.linalg.eigh(M)
    U = math.sqrt(2 * kT / dt) * (V @ (np.sqrt(w)[:, None] * (V.T @ psi)))
    C = U @ U.T / K
    target = 2 * kT / dt * M
    assert np.linalg.norm(C - target) <= 0.02 * np.linalg.norm(target)


def test_pse_real_part_is_positive_definite():
    """The positively split Ewald real-space part is itself SPD (the reason the split
    admits separate square roots)."""
    rng = fsdgen.rng_from(5)
    L = 9.0
    x = rng.random((6, 3)) * L
    for xi in (0.6, 1.0):
        Mr = pse.real_mobility(x, L, 1.0, 1.0, xi, 3.6 / xi)
        w = np.linalg.eigvalsh(0.5 * (Mr + Mr.T))
        assert np.abs(Mr - Mr.T).max() < 1e-13
        assert w.min() > 0


def test_near_field_force_vanishes_without_pairs_and_is_momentum_free():
    rng = fsdgen.rng_from(6)
    shapes = [fsdgen.sticking_cluster(rng, 4) for _ in range(5)]
    com, quat = fsdgen.place_clusters(rng, shapes, 12.0, gap=0.02)
    offsets = np.r_[0, np.cumsum([len(s) for s in shapes])]
    xb = rigid.centre_bodies(np.concatenate(shapes), offsets)
    x = com[rigid.body_index(offsets)] + rigid.bead_vectors(quat, xb, offsets)
    body = rigid.body_index(offsets)
    psi = rng.normal(size=(len(x), 3))
    f0 = brownian.near_field_force(x, body, 12.0, 1.0, 1.0, 0.0, psi, 1.0, 1.0)
    assert np.all(f0 == 0)
    f = brownian.near_field_force(x, body, 12.0, 1.0, 1.0, 3.0, psi, 1.0, 1.0)
    # R_nf annihilates uniform translations, so its square root sums to zero force; the
    # square root of rounding-level eigenvalues (1e-16 of the largest) leaves ~1e-8
    assert np.abs(f.sum(axis=0)).max() < 1e-6 * np.abs(f).max()


def test_lanczos_root_one_step_closed_form():
    """One Lanczos step: |z| V_1 T_1^{1/2} e_1 = sqrt(z^T A z / z^T z) z."""
    rng = np.random.default_rng(11)
    B = rng.normal(size=(9, 9))
    A = B @ B.T + 0.3 * np.eye(9)
    z = rng.normal(size=9)
    got = brownian.lanczos_sqrt_apply(A, z, 1)
    assert np.allclose(got, math.sqrt(z @ A @ z / (z @ z)) * z, rtol=1e-13, atol=0)


def test_lanczos_root_exact_on_invariant_krylov_space():
    """A matrix with m distinct eigenvalues has a Krylov space of dimension m: the m-step
    root is the exact one, and more steps stop there (the basis exhausts the space).  The
    zero eigenvalue comes out of T_k as a rounding-sized Ritz value whose square root is
    about 1e-8 of the scale, which sets the tolerance."""
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.normal(size=(15, 15)))
    lam = np.repeat([0.0, 0.4, 2.5, 9.0], [3, 4, 4, 4])  # singular, like the lubrication matrix
    A = (Q * lam) @ Q.T
    z = rng.normal(size=15)
    exact = brownian.sqrt_apply(A, z)
    for k in (4, 5, 15):
        assert np.linalg.norm(brownian.lanczos_sqrt_apply(A, z, k) - exact) < 1e-7 * np.linalg.norm(exact), k
    assert np.linalg.norm(brownian.lanczos_sqrt_apply(A, z, 3) - exact) > 1e-3 * np.linalg.norm(exact)


def test_lanczos_root_full_space_and_monotone_convergence():
    """With as many steps as the dimension the root is exact for a generic SPD matrix; on the
    way there the error of the Krylov approximation shrinks."""
    rng = np.random.default_rng(13)
    B = rng.normal(size=(20, 20))
    A = B @ B.T + 0.05 * np.eye(20)
    z = rng.normal(size=20)
    exact = brownian.sqrt_apply(A, z)
    errs = [np.linalg.norm(brownian.lanczos_sqrt_apply(A, z, k) - exact) for k in (2, 6, 12, 20)]
    assert errs[-1] < 1e-10 * np.linalg.norm(exact)
    assert errs[0] > errs[1] > errs[2] > errs[3]


def test_near_field_force_with_lanczos_steps_approaches_exact():
    """The near-field force with k Lanczos steps tends to the exact root as k grows (a small
    doublet pair, whose lubrication matrix is singular)."""
    x = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [4.05, 0.3, 0.0], [6.0, 0.6, 0.2]])
    body = np.array([0, 0, 1, 1])
    psi = np.random.default_rng(14).normal(size=(4, 3))
    ex = brownian.near_field_force(x, body, 30.0, 1.0, 1.0, 3.0, psi, 1.0, 1e-3)
    e = [np.linalg.norm(brownian.near_field_force(x, body, 30.0, 1.0, 1.0, 3.0, psi, 1.0, 1e-3, lanczos_steps=k) - ex)
         for k in (1, 3, 12)]
    assert e[2] < 1e-6 * np.linalg.norm(ex) and e[0] > e[2]
