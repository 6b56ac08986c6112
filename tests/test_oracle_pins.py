"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage or the mathematics that fixes the expected value.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import spherical_jn

from oracle import integrate, lub, rigid, rpy, saddle

A, ETA = 1.0, 1.0


# --------------------------------------------------------------------------
# Hasimoto: periodic single-bead mobility (Section 3.1.3 uses 1 + 2.84 R_h/L)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L", [8.0, 16.0, 32.0])
@pytest.mark.parametrize("xi", [0.4, 0.8])
def test_hasimoto_single_bead(L, xi):
    M = rpy.periodic_mobility(np.zeros((1, 3)), L, A, ETA, xi=xi)
    ht, hr = rpy.hasimoto_self(L, A, ETA)
    assert np.allclose(np.diag(M)[:3], ht, rtol=1e-12, atol=0)
    assert np.allclose(np.diag(M)[3:], hr, rtol=1e-12, atol=0)
    assert np.abs(M - np.diag(np.diag(M))).max() < 1e-15
    # the paper's rounded constant: R_h(L) / R_h(inf) = 1 + 2.84 R_h / L to O((a/L)^3)
    assert abs(rpy.HASIMOTO - 2.84) < 5e-3


# --------------------------------------------------------------------------
# closed-form FT-RPY blocks against the spectral radial integrals
# --------------------------------------------------------------------------

def _radial(psi, F, r, ab_g, PQ, k0=3.0):
    """int_0^inf psi(k) F(k r) dk.

    [0, k0]: direct quadrature.  [k0, inf): psi = alpha + beta cos(2ak) +
    gamma sin(2ak) and F(kr) = P sin(kr) + Q cos(kr) are multiplied out into
    single-frequency terms, each integrated with a Fourier-weighted rule.
    """
    head = quad(lambda k: psi(k) * F(k * r), 0.0, k0, limit=400, epsabs=1e-15, epsrel=1e-13)[0]
    al, be, ga = ab_g
    Pf, Qf = PQ
    terms = [
        (lambda k: al(k) * Pf(k), "sin", r), (lambda k: al(k) * Qf(k), "cos", r),
        (lambda k: 0.5 * be(k) * Pf(k), "sin", r + 2 * A), (lambda k: 0.5 * be(k) * Pf(k), "sin", r - 2 * A),
        (lambda k: 0.5 * be(k) * Qf(k), "cos", r + 2 * A), (lambda k: 0.5 * be(k) * Qf(k), "cos", r - 2 * A),
        (lambda k: 0.5 * ga(k) * Pf(k), "cos", r - 2 * A), (lambda k: -0.5 * ga(k) * Pf(k), "cos", r + 2 * A),
        (lambda k: 0.5 * ga(k) * Qf(k), "sin", r + 2 * A), (lambda k: -0.5 * ga(k) * Qf(k), "sin", r - 2 * A),
    ]
    tail = 0.0
    for f, kind, w in terms:
        if abs(w) < 1e-14:
            if kind == "cos":
                tail += quad(f, k0, np.inf, limit=400)[0]
            continue
        sgn = -1.0 if (kind == "sin" and w < 0) else 1.0
        tail += sgn * quad(f, k0, np.inf, weight=kind, wvar=abs(w))[0]
    return head + tail


def _spectral_rpy(r):
    """(tI, tR, rI, rR, c) from the spectral definition (Section 2.2 far-field M)."""
    y = lambda k: k * A
    sinc = lambda k: spherical_jn(0, y(k))
    jv = lambda k: 3.0 * spherical_jn(1, y(k)) / y(k)
    FI = lambda x: spherical_jn(0, x) - spherical_jn(1, x) / x
    FR = lambda x: spherical_jn(2, x)
    Fc = lambda x: spherical_jn(1, x)
    # trig forms: F_I = sin x (1/x - 1/x^3) + cos x / x^2,  F_R = sin x (3/x^3 - 1/x) - 3 cos x / x^2,
    # j1 = sin x / x^2 - cos x / x
    PQ_I = (lambda k: 1 / (k * r) - 1 / (k * r) ** 3, lambda k: 1 / (k * r) ** 2)
    PQ_R = (lambda k: 3 / (k * r) ** 3 - 1 / (k * r), lambda k: -3 / (k * r) ** 2)
    PQ_c = (lambda k: 1 / (k * r) ** 2, lambda k: -1 / (k * r))
    # psi_tt = sinc^2 = (1 - cos 2y) / (2 y^2)
    tt_abg = (lambda k: 1 / (2 * y(k) ** 2), lambda k: -1 / (2 * y(k) ** 2), lambda k: 0.0)
    # psi_rr = k^2 jv^2 / 4, jv^2 = (9/y^6)[(1+y^2)/2 + (y^2-1)/2 cos 2y - y sin 2y]
    rr_abg = (lambda k: k * k / 4 * 9 / y(k) ** 6 * 0.5 * (1 + y(k) ** 2),
              lambda k: k * k / 4 * 9 / y(k) ** 6 * 0.5 * (y(k) ** 2 - 1),
              lambda k: -k * k / 4 * 9 / y(k) ** 6 * y(k))
    # psi_rt = k sinc jv = k (3/y^4)[(1 - cos 2y)/2 - (y/2) sin 2y]
    rt_abg = (lambda k: k * 1.5 / y(k) ** 4, lambda k: -k * 1.5 / y(k) ** 4, lambda k: -k * 1.5 / y(k) ** 3)
    pre = 1.0 / (2 * math.pi ** 2 * ETA)
    tI = pre * _radial(lambda k: sinc(k) ** 2, FI, r, tt_abg, PQ_I)
    tR = pre * _radial(lambda k: sinc(k) ** 2, FR, r, tt_abg, PQ_R)
    rI = pre * _radial(lambda k: k * k / 4 * jv(k) ** 2, FI, r, rr_abg, PQ_I)
    rR = pre * _radial(lambda k: k * k / 4 * jv(k) ** 2, FR, r, rr_abg, PQ_R)
    c = -1.0 / (4 * math.pi ** 2 * ETA) * _radial(lambda k: k * sinc(k) * jv(k), Fc, r, rt_abg, PQ_c)
    return tI, tR, rI, rR, c


@pytest.mark.parametrize("r", [0.35, 0.9, 1.5, 1.95, 2.0, 2.6, 4.3, 7.0])
def test_rpy_closed_forms_match_spectral_integrals(r):
    closed = rpy.rpy_scalars(np.array([r]), A, ETA)
    spec = _spectral_rpy(r)
    scale = (rpy.mu_t(A, ETA), rpy.mu_t(A, ETA), rpy.mu_r(A, ETA), rpy.mu_r(A, ETA),
             1 / (8 * math.pi * ETA * A * A))
    for cval, sval, sc in zip(closed, spec, scale):
        assert abs(float(cval[0]) - sval) < 1e-9 * sc, (r, float(cval[0]), sval)


# --------------------------------------------------------------------------
# Gaussian-damped radial transforms against quadrature
# --------------------------------------------------------------------------

@pytest.mark.parametrize("xi", [0.3, 0.7])
def test_damped_transforms_match_quadrature(xi):
    for m in rpy.beenakker_multipliers(A, xi):
        phi = lambda k: np.polynomial.polynomial.polyval(k * k, m.c) * math.exp(-k * k / (4 * xi * xi))
        kmax = 30 * xi
        for r in (0.5, 1.7, 3.0, 6.5):
            A_q = quad(lambda k: phi(k) * spherical_jn(0, k * r), 0, kmax, limit=400)[0] / (2 * math.pi ** 2)
            S2_q = r * r * quad(lambda k: phi(k) * spherical_jn(1, k * r) / k if k > 0 else 0.0,
                                0, kmax, limit=400)[0] / (2 * math.pi ** 2)
            dA_q = -quad(lambda k: phi(k) * k * spherical_jn(1, k * r), 0, kmax, limit=400)[0] / (2 * math.pi ** 2)
            sc = abs(quad(lambda k: abs(phi(k)), 0, kmax)[0]) / (2 * math.pi ** 2)
            assert abs(m.A(np.array(r)) - A_q) < 1e-11 * sc
            assert abs(m.S2(np.array(r)) - S2_q) < 1e-11 * sc * r ** 3
            assert abs(m.dA(np.array(r)) - dA_q) < 1e-11 * sc
        a0 = quad(phi, 0, kmax)[0] / (2 * math.pi ** 2)
        assert abs(m.A0() - a0) < 1e-12 * abs(a0)


# --------------------------------------------------------------------------
# splitting-parameter invariance, symmetry, positive definiteness
# --------------------------------------------------------------------------

def _random_beads(n, L, seed, min_gap=2.05):
    rng = np.random.default_rng(seed)
    x = []
    while len(x) < n:
        p = rng.random(3) * L
        ok = True
        for q in x:
            d = p - q
            d -= L * np.round(d / L)
            if np.linalg.norm(d) < min_gap:
                ok = False
                break
        if ok:
            x.append(p)
    return np.array(x)


def test_xi_invariance():
    x = _random_beads(8, 10.0, 1)
    M1 = rpy.periodic_mobility(x, 10.0, A, ETA, xi=0.35)
    M2 = rpy.periodic_mobility(x, 10.0, A, ETA, xi=0.9)
    assert np.abs(M1 - M2).max() < 1e-12 * np.abs(M1).max()


def test_xi_invariance_with_overlaps_and_images():
    # overlapping beads exercise the r < 2a branch; L small forces many images
    x = np.array([[0.0, 0.0, 0.0], [1.3, 0.2, -0.1], [2.5, 2.6, 0.4]])
    M1 = rpy.periodic_mobility(x, 6.0, A, ETA, xi=0.5)
    M2 = rpy.periodic_mobility(x, 6.0, A, ETA, xi=1.2)
    assert np.abs(M1 - M2).max() < 1e-12 * np.abs(M1).max()


def test_mobility_symmetric_positive_definite():
    x = _random_beads(12, 11.0, 2)
    M = rpy.periodic_mobility(x, 11.0, A, ETA)
    assert np.abs(M - M.T).max() < 1e-14 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0


def test_large_box_approaches_free_space():
    # periodic images shift every tt block by -2.8373 / (6 pi eta L) I at O(1/L)
    L = 400.0
    x = np.array([[0.0, 0.0, 0.0], [2.7, -1.1, 0.8]])
    M = rpy.periodic_mobility(x, L, A, ETA)
    Mf = rpy.rpy_free_matrix(x, A, ETA)
    shift = np.zeros_like(M)
    for i in range(2):
        for j in range(2):
            shift[6 * i:6 * i + 3, 6 * j:6 * j + 3] = -rpy.HASIMOTO / (6 * math.pi * ETA * L) * np.eye(3)
    assert np.abs(M - Mf - shift).max() < 1e-6 * rpy.mu_t(A, ETA)


def test_covariance_under_cubic_rotations():
    x = _random_beads(5, 9.0, 3)
    L = 9.0
    M = rpy.periodic_mobility(x, L, A, ETA, xi=0.6)
    for R in (np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]]), np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0.0]])):
        MR = rpy.periodic_mobility(x @ R.T, L, A, ETA, xi=0.6)
        T = np.kron(np.eye(2 * len(x)), R)
        assert np.abs(MR - T @ M @ T.T).max() < 1e-13 * np.abs(M).max()


# --------------------------------------------------------------------------
# lubrication model
# --------------------------------------------------------------------------

def test_lubrication_vanishes_at_cutoff_and_is_psd():
    assert abs(lub.X_squeeze(1.0)) < 1e-15 and abs(lub.Y_shear(1.0)) < 1e-15
    x = np.array([[0.0, 0, 0], [2.3, 0.1, 0], [4.4, 0.5, 0.2], [0.0, 2.2, 0.0]])
    R = lub.resistance_matrix(x, np.arange(4), 20.0, A, ETA, 3.0)
    assert np.abs(R - R.T).max() < 1e-13
    assert np.linalg.eigvalsh(R).min() > -1e-10


def test_reynolds_squeeze_limit():
    # two single-bead aggregates pushed together: F / dU -> 6 pi eta a / (4 eps)
    for eps in (1e-3, 1e-4):
        L = 30.0
        d = 2 * A + eps * A
        com = np.array([[0.0, 0, 0], [d, 0, 0]])
        quat = np.tile([1.0, 0, 0, 0], (2, 1))
        force = np.zeros((2, 6))
        force[0, 0], force[1, 0] = 1.0, -1.0
        U, *_ = saddle.solve(L, A, ETA, [0, 1, 2], np.zeros((2, 3)), com, quat, force,
                             np.zeros((3, 3)), r_lub=3 * A, eps_min=1e-6)
        dU = U[0, 0] - U[1, 0]
        ratio = (1.0 / dU) / (6 * math.pi * ETA * A / (4 * eps))
        # the log term and the far field add O(eps ln eps) relative corrections
        assert abs(ratio - 1) < 12 * eps * math.log(1 / eps) + 2 * eps


# --------------------------------------------------------------------------
# near-contact asymptotics of two equal spheres (lubrication theory: the squeeze
# resistance grows as 1/(4 eps) + (9/40) ln(1/eps), the sliding one as (1/6) ln(1/eps);
# Jeffrey & Onishi's expansions, which the paper's Section 2.1 lubrication relies on)
# --------------------------------------------------------------------------

def pair_drag(eps, axis):
    """F / (6 pi eta a dU) of two one-bead aggregates at gap eps a, pushed by equal and
    opposite unit forces along `axis` (0: the line of centres, 1: across it)."""
    L = 40.0
    com = np.array([[0.0, 0, 0], [2 * A + eps * A, 0, 0]])
    quat = np.tile([1.0, 0, 0, 0], (2, 1))
    force = np.zeros((2, 6))
    force[0, axis], force[1, axis] = 1.0, -1.0
    U, *_ = saddle.solve(L, A, ETA, [0, 1, 2], np.zeros((2, 3)), com, quat, force,
                         np.zeros((3, 3)), r_lub=3 * A, eps_min=1e-7)
    return 1.0 / (6 * math.pi * ETA * A * (U[0, axis] - U[1, axis]))


def log_coefficients():
    """(squeeze, sliding) log coefficients read off the full solve between the gaps 1e-4 a
    and 1e-5 a: the far field changes by O(1e-4) there, so the differences isolate the
    near-contact terms (the 1/(4 eps) pole is taken out of the squeeze difference)."""
    e1, e2 = 1e-4, 1e-5
    sq = pair_drag(e2, 0) - pair_drag(e1, 0) - 0.25 * (1 / e2 - 1 / e1)
    sl = pair_drag(e2, 1) - pair_drag(e1, 1)
    return sq / math.log(10.0), sl / math.log(10.0)


def test_lubrication_log_coefficients():
    sq, sl = log_coefficients()
    assert abs(sq - 9 / 40) < 1e-3
    assert abs(sl - 1 / 6) < 1e-3


@pytest.mark.parametrize("which,bad", [("Y_shear", lambda e: np.log(1 / np.asarray(e, float)) / 4),
                                       ("X_squeeze", lambda e: 0.25 / np.asarray(e, float) + 0.3 * np.log(1 / np.asarray(e, float)) - 0.25)])
def test_log_coefficient_pin_catches_a_wrong_coefficient(monkeypatch, which, bad):
    # a mistake planted in the oracle (1/4 for 1/6, 3/10 for 9/40) must fail the pin above
    monkeypatch.setattr(lub, which, bad)
    sq, sl = log_coefficients()
    assert abs(sq - 9 / 40) > 1e-2 or abs(sl - 1 / 6) > 1e-2


def _sheared_pair(eps):
    """Two three-bead aggregates whose only inter-body pair (bead 0 of each) sits at gap
    eps a along n = (1, 1, 0)/sqrt(2), in simple shear u_x = y.  Returns the lab-frame
    rate at which that gap closes, (u_p - u_q) . n with u = U + Omega x r, and the rate
    affine motion with the flow would give, n . G d."""
    n = np.array([1.0, 1.0, 0.0]) / math.sqrt(2)
    d = (2 + eps) * A
    arm = np.array([[0.0, 0, 0], [-2.0, 0, 0], [-2.0, 0, 2.0]])     # bead 0 at the tip
    xb = np.concatenate([arm, -arm])    # body 0 reaches towards -x, body 1 towards +x
    X = np.array([arm.mean(0),          # bead 0 of body 0 at the origin
                  d * n - arm.mean(0)])  # bead 0 of body 1 at d n
    G = np.zeros((3, 3))
    G[0, 1] = 1.0
    quat = np.tile([1.0, 0, 0, 0], (2, 1))
    U, _, _, asm = saddle.solve(40.0, A, ETA, [0, 3, 6], xb, X, quat, np.zeros((2, 6)), G,
                                r_lub=3 * A, eps_min=1e-7)
    pairs_ = lub.pairs(asm.x, rigid.body_index([0, 3, 6]), 40.0, 3 * A)
    assert len(pairs_[0]) == 1 and (pairs_[0][0], pairs_[1][0]) == (0, 3)
    u = U[rigid.body_index([0, 3, 6]), :3] + np.cross(U[rigid.body_index([0, 3, 6]), 3:], asm.r)
    dd = asm.x[0] - asm.x[3]
    return (u[0] - u[3]) @ n, n @ G @ dd


def test_sheared_pair_stops_closing_at_contact():
    # R_FE : E_inf (Eq. `FH_agg`) read as the pair force on the lab-frame closing rate: the
    # gap of a near-touching inter-body pair closes at a rate that vanishes like 1/X(eps),
    # however fast the shear would bring the two bodies together
    r4, a4 = _sheared_pair(1e-4)
    r5, a5 = _sheared_pair(1e-5)
    assert abs(a4) > 0.4 and abs(a5) > 0.4
    assert abs(r4 / a4) < 2e-3 and abs(r5 / a5) < 2e-4
    assert 0.05 < (r5 / a5) / (r4 / a4) < 0.2


def test_sheared_pair_pin_catches_a_flipped_strain_term(monkeypatch):
    # planted in the oracle: the bead-level strain force with the wrong sign, or left out
    real = lub.strain_forces
    for scale in (-1.0, 0.0):
        monkeypatch.setattr(lub, "strain_forces", lambda *a, _s=scale, **k: _s * real(*a, **k))
        r5, a5 = _sheared_pair(1e-5)
        assert abs(r5 / a5) > 0.1


def test_ambient_rotation_moves_bodies_rigidly():
    # a purely rotational ambient flow carries every body with it: U = (W X, Omega_inf)
    # with no lubrication force, whatever the gaps
    rng = np.random.default_rng(11)
    xb = np.concatenate([rng.normal(size=(3, 3)), rng.normal(size=(3, 3))])
    com = np.array([[0.0, 0, 0], [2.6, 0.3, -0.2]])
    quat = np.tile([1.0, 0, 0, 0], (2, 1))
    Wm = np.array([[0.0, -0.7, 0.2], [0.7, 0.0, -0.4], [-0.2, 0.4, 0.0]])
    U, _, _, asm = saddle.solve(30.0, A, ETA, [0, 3, 6], xb * 0.8, com, quat, np.zeros((2, 6)), Wm,
                                r_lub=3 * A)
    E, W = rigid.strain_and_spin(Wm)
    assert np.allclose(U[:, :3], asm.com @ Wm.T, atol=1e-12)
    assert np.allclose(U[:, 3:], W, atol=1e-12)


# --------------------------------------------------------------------------
# rigid-body constraint and solves
# --------------------------------------------------------------------------

def test_sigma_matches_cross_products():
    rng = np.random.default_rng(4)
    r = rng.normal(size=(5, 3))
    offs = [0, 2, 5]
    S = rigid.sigma_matrix(r, offs)
    lam = rng.normal(size=(5, 6))
    out = (S @ lam.reshape(-1)).reshape(2, 6)
    for j, (s, e) in enumerate(((0, 2), (2, 5))):
        assert np.allclose(out[j, :3], lam[s:e, :3].sum(0))
        assert np.allclose(out[j, 3:], (lam[s:e, 3:] + np.cross(r[s:e], lam[s:e, :3])).sum(0))
    V = rng.normal(size=(2, 6))
    u = (S.T @ V.reshape(-1)).reshape(5, 6)
    for i, j in enumerate([0, 0, 1, 1, 1]):
        assert np.allclose(u[i, :3], V[j, :3] + np.cross(V[j, 3:], r[i]))
        assert np.allclose(u[i, 3:], V[j, 3:])


def test_single_bead_aggregates_reduce_to_mobility_matvec():
    x = _random_beads(6, 12.0, 5)
    rng = np.random.default_rng(6)
    force = rng.normal(size=(6, 6))
    U, F, res, Asm = saddle.solve(12.0, A, ETA, np.arange(7), np.zeros((6, 3)), x,
                                  np.tile([1.0, 0, 0, 0], (6, 1)), force, np.zeros((3, 3)))
    M = rpy.periodic_mobility(rigid.wrap(x, 12.0), 12.0, A, ETA)
    assert np.abs(U.reshape(-1) - M @ force.reshape(-1)).max() < 1e-12 * np.abs(U).max()
    assert res < 1e-13


def _small_system(seed=7, shear=True, lubr=True):
    import fsdgen
    rng = fsdgen.rng_from(seed)
    shapes = [fsdgen.sticking_cluster(rng, nb) for nb in (3, 5, 1, 4)]
    L = 12.0
    com, quat = fsdgen.place_clusters(rng, shapes, L, gap=0.05)
    offs = np.r_[0, np.cumsum([len(s) for s in shapes])]
    return dict(L=L, a=A, eta=ETA, offsets=offs, x_body=np.concatenate(shapes), com=com, quat=quat,
                force=rng.normal(size=(4, 6)),
                grad_u=fsdgen.simple_shear(1.0) if shear else np.zeros((3, 3)),
                r_lub=3.0 if lubr else 0.0)


def test_solve_routes_agree():
    kw = _small_system()
    Asm = saddle.assemble(**kw)
    F1, V1 = saddle.solve_schur(Asm)
    F2, V2 = saddle.solve_lu(Asm)
    K, b = saddle.saddle_matrix(Asm), saddle.rhs(Asm)
    P = saddle.preconditioner(Asm, kw["offsets"], A, ETA, kw["L"])
    x, its, rr = saddle.gmres(K, b, P, tol=1e-13, restart=40)
    n1 = len(F1)
    assert np.abs(V1 - V2).max() < 1e-11 * np.abs(V1).max()
    assert np.abs(x[n1:] - V1).max() < 1e-9 * np.abs(V1).max()
    assert saddle.residual(Asm, F1, V1) < 1e-13
    # the preconditioner must help: fewer iterations than unpreconditioned GMRES
    _, its0, _ = saddle.gmres(K, b, None, tol=1e-13, restart=40, maxit=4000)
    assert its < its0


def test_linearity_in_forcing():
    kw = _small_system()
    f1 = kw["force"]
    U_f, *_ = saddle.solve(**{**kw, "grad_u": np.zeros((3, 3))})
    U_s, *_ = saddle.solve(**{**kw, "force": np.zeros_like(f1)})
    U_fs, *_ = saddle.solve(**kw)
    U_2f, *_ = saddle.solve(**{**kw, "force": 2 * f1, "grad_u": np.zeros((3, 3))})
    sc = np.abs(U_fs).max()
    assert np.abs(U_fs - (U_f + U_s)).max() < 1e-11 * sc
    assert np.abs(U_2f - 2 * U_f).max() < 1e-11 * sc


def test_aggregate_mobility_reciprocal_and_positive():
    kw = _small_system(shear=False)
    na = len(kw["offsets"]) - 1
    cols = []
    for m in range(6 * na):
        f = np.zeros(6 * na)
        f[m] = 1.0
        U, *_ = saddle.solve(**{**kw, "force": f.reshape(na, 6)})
        cols.append(U.reshape(-1))
    N = np.array(cols).T
    assert np.abs(N - N.T).max() < 1e-11 * np.abs(N).max()
    assert np.linalg.eigvalsh(0.5 * (N + N.T)).min() > 0


def test_translation_invariance_without_shear():
    kw = _small_system(shear=False)
    U1, *_ = saddle.solve(**kw)
    U2, *_ = saddle.solve(**{**kw, "com": kw["com"] + np.array([1.3, -4.1, 2.2])})
    assert np.abs(U1 - U2).max() < 1e-11 * np.abs(U1).max()


def test_identical_centrosymmetric_pair_settles_equally():
    # Section 3.1.2: two identical bodies settle with identical velocities.
    # Point inversion about the box centre maps the pair onto itself with the
    # forces reversed, so U_A = U_B and W_A = -W_B.
    xb = np.array([[-1.0, 0, 0], [1.0, 0, 0], [-1.0, 0, 0], [1.0, 0, 0]])
    q = np.array([0.9, 0.1, -0.3, 0.2])
    quat = np.tile(q / np.linalg.norm(q), (2, 1))
    com = np.array([[1.2, 0.7, 2.9], [-1.2, -0.7, -2.9]])
    force = np.zeros((2, 6))
    force[:, 2] = -1.0
    U, *_ = saddle.solve(20.0, A, ETA, [0, 2, 4], xb, com, quat, force, np.zeros((3, 3)))
    assert np.abs(U[0, :3] - U[1, :3]).max() < 1e-12
    assert np.abs(U[0, 3:] + U[1, 3:]).max() < 1e-12


def test_doublet_in_shear_has_cos2theta_form():
    # Section 3.1.1: omega_z / gamma = -1/2 (1 + B cos 2 theta); B is not fixed at
    # force-torque RPY level, the functional form is.
    L = 60.0
    ths = np.linspace(0, math.pi, 7, endpoint=False)
    om = []
    for th in ths:
        q = np.array([math.cos(th / 2), 0, 0, math.sin(th / 2)])   # rotate body x into the xy plane
        U, *_ = saddle.solve(L, A, ETA, [0, 2], np.array([[-1.0, 0, 0], [1.0, 0, 0]]),
                             np.zeros((1, 3)), q[None], np.zeros((1, 6)), np.array([[0, 1.0, 0], [0, 0, 0], [0, 0, 0]]))
        om.append(U[0, 5])
    om = np.array(om)
    Afit = np.stack([np.ones_like(ths), np.cos(2 * ths), np.sin(2 * ths)], 1)
    coef, *_ = np.linalg.lstsq(Afit, om, rcond=None)
    assert np.abs(Afit @ coef - om).max() < 1e-4
    assert abs(coef[0] + 0.5) < 0.02      # mean rotation -gamma/2 up to lattice corrections
    assert 0 < -coef[1] / 0.5 < 1.0 or 0 < coef[1] / 0.5 < 1.0


# --------------------------------------------------------------------------
# time integration
# --------------------------------------------------------------------------

def test_quaternion_update_converges_to_rigid_rotation():
    om = np.array([0.3, -0.2, 0.5])
    T = 1.0
    errs = []
    for n in (200, 400):
        q = np.array([[1.0, 0, 0, 0]])
        X = np.zeros((1, 3))
        for _ in range(n):
            X, q = integrate.euler_step(X, q, np.r_[0, 0, 0, om][None], T / n, 100.0)
        ang = np.linalg.norm(om) * T
        ax = om / np.linalg.norm(om)
        exact = np.r_[math.cos(ang / 2), math.sin(ang / 2) * ax]
        errs.append(np.abs(q[0] - exact).max())
    assert errs[1] < 0.6 * errs[0] and errs[1] < 1e-3
    assert abs(np.linalg.norm(q) - 1) < 1e-14
    R = rigid.rotation_matrix(q)[0]
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-13) and abs(np.linalg.det(R) - 1) < 1e-13
