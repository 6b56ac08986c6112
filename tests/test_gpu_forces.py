"""Conservative bead-pair forces on the GPU (Section 4.2) through the C ABI.

- the bead forces (Hertz contact, regularised van der Waals, double layer) against the
  oracle's brute-force pair sum, with overlapping and near-contact pairs and periodic images;
- a saddle solve with the forces switched on against the oracle's solve with the same
  forces summed into each body (Sigma);
- two beads pressed together by opposite loads come to rest where the Hertz force balances
  the load, r = 2a - (F/k_n)^(2/3).
"""
import numpy as np
import pytest

import fsdgen
from oracle import forces, rigid, saddle

pytestmark = pytest.mark.gpu

COEF = dict(k_n=200.0, hamaker=0.8, Z=3.0, kappa=1.5, h_c=0.05)


@pytest.fixture(scope="module")
def F(gpu):
    import paper_2607_25161_amd as F
    return F


def _system(seed=41, L=9.0):
    """Single beads in close pairs (overlaps down to r = 1.6 a, gaps up to 0.9 a) and a few
    clusters, in a small box so that pairs also meet through the faces.  Every other bead
    pair is kept at least 2.2 a apart."""
    rng = fsdgen.rng_from(seed)
    shapes = [fsdgen.sticking_cluster(rng, nb) for nb in (4, 3, 5)]
    com, quat = fsdgen.place_clusters(rng, shapes, L, gap=0.3)
    offs0 = np.r_[0, np.cumsum([len(x) for x in shapes])].astype(np.int32)
    xb0 = rigid.centre_bodies(np.concatenate(shapes), offs0)
    placed = list(com[rigid.body_index(offs0)] + rigid.bead_vectors(quat, xb0, offs0))

    def far(p):
        d = np.array(placed) - p
        d -= L * np.round(d / L)
        return np.linalg.norm(d, axis=1).min() >= 2.2

    def wrap(p):
        return (p + L / 2) % L - L / 2

    singles = []
    for r in (1.6, 1.85, 1.99, 2.02, 2.3, 2.9, None):  # None: a pair 1.8 a apart through the x face
        for _ in range(10000):
            if r is None:
                y, z = rng.uniform(-L / 2, L / 2, 2)
                p1, p2 = np.array([L / 2 - 0.3, y, z]), wrap(np.array([L / 2 + 1.5, y + 0.1, z - 0.1]))
            else:
                c = rng.uniform(-L / 2, L / 2, 3)
                d = rng.normal(size=3)
                p1, p2 = c, wrap(c + r * d / np.linalg.norm(d))
            if far(p1) and far(p2):
                break
        else:
            raise RuntimeError("placement failed")
        placed += [p1, p2]
        singles += [p1, p2]
    xb = shapes + [np.zeros((1, 3))] * len(singles)
    com = np.vstack([com, np.array(singles)])
    quat = np.vstack([quat, np.tile([1.0, 0, 0, 0], (len(singles), 1))])
    offs = np.r_[0, np.cumsum([len(x) for x in xb])].astype(np.int32)
    return dict(L=L, a=1.0, eta=1.0, offsets=offs, x_body=np.concatenate(xb), com=com, quat=quat,
                force=rng.normal(size=(len(xb), 6)), grad_u=fsdgen.simple_shear(1.0), r_lub=0.0)


def _make(F, kw, **p):
    par = dict(xi=0.6, ewald_tol=1e-10, r_lub=0.0, r_precond=0.0, gmres_tol=1e-11, gmres_restart=40,
               gmres_maxit=4000)
    par.update(p)
    s = F.System(F.default_params(**par))
    s.init_box(kw["L"])
    s.init_aggregates(kw["offsets"], kw["x_body"], kw["com"], kw["quat"])
    s.set_forces(kw["force"])
    s.set_shear(kw["grad_u"])
    return s


def test_pair_forces_match_oracle(F):
    kw = _system()
    s = _make(F, kw)
    assert np.abs(s.pair_forces()).max() == 0  # off by default
    s.set_pair_forces(r_cut=3.0, **{k: v for k, v in COEF.items()})
    f = s.pair_forces()
    A = saddle.assemble(**kw)
    body = rigid.body_index(kw["offsets"])
    ref = forces.bead_forces(A.x, body, kw["L"], 1.0, 3.0, **COEF)
    assert np.abs(ref).max() > 1.0  # contact and near-contact pairs present
    assert np.abs(f - ref).max() <= 1e-12 * np.abs(ref).max()
    # each family alone
    for part in (dict(k_n=COEF["k_n"]), dict(hamaker=COEF["hamaker"], h_c=COEF["h_c"]),
                 dict(Z=COEF["Z"], kappa=COEF["kappa"])):
        s.set_pair_forces(r_cut=2.5, **part)
        ref = forces.bead_forces(A.x, body, kw["L"], 1.0, 2.5, **part)
        assert np.abs(s.pair_forces() - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300), part
    s.close()


def test_pair_force_arguments_checked(F):
    kw = _system()
    s = _make(F, kw)
    for bad in (dict(k_n=-1.0), dict(hamaker=1.0, h_c=0.0), dict(Z=1.0, kappa=0.0), dict(k_n=1.0, r_cut=1.5),
                dict(k_n=1.0, r_cut=1e3)):
        with pytest.raises(F.FsdError):
            s.set_pair_forces(**bad)
    s.close()


def test_solve_with_pair_forces_matches_oracle(F):
    kw = _system(seed=42)
    s = _make(F, kw)
    s.set_pair_forces(r_cut=3.0, **COEF)
    U, _, info = s.solve()
    A = saddle.assemble(**kw)
    body = rigid.body_index(kw["offsets"])
    fb = forces.bead_forces(A.x, body, kw["L"], 1.0, 3.0, **COEF)
    lam = np.zeros((len(fb), 6))
    lam[:, :3] = fb
    ft = kw["force"] + (A.Sig @ lam.reshape(-1)).reshape(-1, 6)
    Uo, *_ = saddle.solve(**{**kw, "force": ft})
    for sl in (slice(0, 3), slice(3, 6)):
        assert np.linalg.norm(U[:, sl] - Uo[:, sl]) <= 1e-8 * np.linalg.norm(Uo[:, sl])
    s.close()


def test_contact_force_balances_a_pushing_load(F):
    """Two beads pressed together by opposite loads +-F come to rest where the Hertz force
    balances the load, r = 2a - (F/k_n)^(2/3) (at rest the hydrodynamic forces vanish);
    without the contact force they run into each other until the overlap check stops them."""
    L, load, kn = 20.0, 10.0, 1e3
    kw = dict(L=L, offsets=np.array([0, 1, 2], dtype=np.int32), x_body=np.zeros((2, 3)),
              com=np.array([[-1.0, 0.0, 0.0], [1.0, 0.0, 0.0]]), quat=np.tile([1.0, 0, 0, 0], (2, 1)),
              force=np.array([[load, 0, 0, 0, 0, 0], [-load, 0, 0, 0, 0, 0]]), grad_u=np.zeros((3, 3)))
    s = _make(F, kw, xi=0.5, ewald_tol=1e-6, gmres_tol=1e-10)
    s.set_pair_forces(k_n=kn, r_cut=2.5)
    for _ in range(300):
        assert s.step(0.005, 1).status == 0
    X, _ = s.state()
    r = X[1, 0] - X[0, 0]
    assert abs(r - (2.0 - (load / kn) ** (2.0 / 3.0))) < 1e-6, r
    assert np.abs(X[:, 1:]).max() < 1e-5  # no drift off the line of centres (to the Ewald tolerance)
    s.close()
    s = _make(F, kw, xi=0.5, ewald_tol=1e-6, gmres_tol=1e-10)
    # the overlapping-bead mobility slows the approach in proportion to r, so this takes
    # several time units
    with pytest.raises(F.FsdError) as e:
        for _ in range(2000):
            s.step(0.005, 1)
    assert e.value.code == -6  # FSD_EOVERLAP
    s.close()
