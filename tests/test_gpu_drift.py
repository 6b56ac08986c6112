"""Brownian drift on the GPU (Appendix A): random finite differences (Eq. `rfd`) and
Fixman's midpoint scheme.

- the drift for a given dq against the oracle's two dense saddle solves at the displaced
  configurations, with and without lubrication;
- a time step with the drift on moves the bodies by (U + drift) dt, with U the saddle
  solve's velocities and the drift that of the step's own dq;
- the batched step applies each system's drift as the single-system step does;
- a step with Fixman's drift moves the bodies by (U + (m/2)(U' - U0)) dt, against the
  oracle's two dense solves with the Brownian terms the library drew.
"""
import numpy as np
import pytest

import fsdgen
from oracle import drift, integrate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F(gpu):
    import paper_2607_25161_amd as F
    return F


def _system(seed=31, sizes=(3, 4, 1, 5, 2), L=11.0, lub_on=True):
    rng = fsdgen.rng_from(seed)
    shapes = [fsdgen.sticking_cluster(rng, nb) for nb in sizes]
    com, quat = fsdgen.place_clusters(rng, shapes, L, gap=0.1)
    offs = np.r_[0, np.cumsum([len(s) for s in shapes])].astype(np.int32)
    return dict(L=L, a=1.0, eta=1.0, offsets=offs, x_body=np.concatenate(shapes), com=com, quat=quat,
                force=np.zeros((len(sizes), 6)), grad_u=np.zeros((3, 3)), r_lub=3.0 if lub_on else 0.0)


def _make(F, kw, **p):
    par = dict(xi=0.6, ewald_tol=1e-10, r_lub=kw["r_lub"], r_precond=2.1 if kw["r_lub"] else 0.0,
               gmres_tol=1e-12, gmres_restart=40, gmres_maxit=4000, kT=0.7)
    par.update(p)
    s = F.System(F.default_params(**par))
    s.init_box(kw["L"])
    s.init_aggregates(kw["offsets"], kw["x_body"], kw["com"], kw["quat"])
    s.set_forces(kw["force"])
    s.set_shear(kw["grad_u"])
    return s


@pytest.mark.parametrize("lub_on", [False, True])
def test_drift_matches_oracle(F, lub_on):
    kw = _system(lub_on=lub_on)
    s = _make(F, kw)
    eps = 1e-3
    s.set_drift(0, eps)  # eps only; the drift below is computed on request
    dq = np.random.default_rng(32).normal(size=(len(kw["offsets"]) - 1, 6))
    d = s.rfd_drift(dq)
    ref = drift.rfd_drift(kw["L"], 1.0, 1.0, kw["offsets"], kw["x_body"], kw["com"], kw["quat"], dq, eps, 0.7,
                          r_lub=kw["r_lub"])
    assert np.abs(ref).max() > 0
    assert np.linalg.norm(d - ref) <= 1e-6 * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)
    X, q = s.state()  # the drift leaves the configuration as it found it
    X0 = (np.asarray(kw["com"]) + kw["L"] / 2) % kw["L"] - kw["L"] / 2
    assert np.abs(X - X0).max() < 1e-12
    s.close()


def test_step_adds_the_drift(F):
    kw = _system(seed=33)
    s = _make(F, kw)
    s.set_brownian(1e-3, step=5)
    na = len(kw["offsets"]) - 1
    nb = int(kw["offsets"][-1])
    s.set_noise(psi_w=np.zeros(3 * s.info().grid ** 3), psi_r=np.zeros(6 * nb), psi_nf=np.zeros(3 * nb))
    U, _, _ = s.solve()        # no Brownian terms (zero noise): the solve's velocities
    dr = s.rfd_drift()         # the drift for the next step's dq
    X0, q0 = s.state()
    s.set_drift(1)
    s.set_brownian(1e-3, step=5)
    s.step(1e-3, 1)
    X1, q1 = s.state()
    Xo, qo = integrate.euler_step(X0, q0, U + dr, 1e-3, kw["L"])
    assert np.abs(X1 - Xo).max() < 1e-12 and np.abs(q1 - qo).max() < 1e-12
    assert np.abs(dr).max() * 1e-3 > 1e-9  # the drift moved the bodies measurably
    s.close()


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("fused", [True, False])
def test_batched_step_with_drift_equals_solo(F, mode, fused):
    """The batched step applies each system's drift as fsd_step does: two Brownian time steps
    of three systems in one batch (multi-system launches or one stream per system) end where
    the same systems end stepped alone, with the same noise (seed, stream, step)."""
    kws = [_system(seed=34 + k, sizes=(3, 2, 4), L=10.0) for k in range(3)]
    par = dict(kT=1.0, gmres_tol=1e-11)
    solo = []
    for kw in kws:
        s = _make(F, kw, **par)
        s.set_drift(mode)
        s.step(1e-3, 2)
        solo.append(s.state())
        s.close()
    live = [_make(F, kw, **par) for kw in kws]
    for s in live:
        s.set_drift(mode)
    b = F.Batch(1 << 34, 4)
    b.set_fused(fused)
    slots = [b.admit(s) for s in live]
    for _ in range(2):
        assert b.step(1e-3) == 0
    for k, s in enumerate(live):
        assert b.info(slots[k]).status == 0
        X, q = s.state()
        # the same arithmetic but for the summation order of the multi-system launches
        assert np.abs(X - solo[k][0]).max() < 1e-11 and np.abs(q - solo[k][1]).max() < 1e-11, k
    b.close()
    for s in live:
        s.close()


def test_fixman_step_matches_oracle(F):
    """A step with Fixman's midpoint drift: the library's update equals the oracle's Euler
    update with U + (m/2)(U' - U0), the oracle taking U0 and U' from its dense solves with the
    Brownian terms the library drew."""
    kw = _system(seed=35)
    s = _make(F, kw)
    dt, m = 1e-3, 100.0
    nb = int(kw["offsets"][-1])
    rng = np.random.default_rng(36)
    s.set_brownian(dt, step=3)
    s.set_noise(psi_w=np.zeros(3 * s.info().grid ** 3), psi_r=rng.normal(size=6 * nb), psi_nf=rng.normal(size=3 * nb))
    U, _, _ = s.solve()
    ub, fb, _ = s.brownian_terms()
    X0, q0 = s.state()
    s.set_drift(2, m)
    s.step(dt, 1)
    X1, q1 = s.state()
    d = drift.fixman_drift(kw["L"], 1.0, 1.0, kw["offsets"], kw["x_body"], kw["com"], kw["quat"], ub, fb, m, dt,
                           r_lub=kw["r_lub"])
    Xo, qo = integrate.euler_step(X0, q0, U + d, dt, kw["L"])
    Xn, qn = integrate.euler_step(X0, q0, U, dt, kw["L"])
    # the drift moves the bodies measurably; the library's move agrees with the oracle's to a
    # small fraction of it ((m/2) amplifies the solves' common error, which mostly cancels)
    for got, want, base in ((X1, Xo, Xn), (q1, qo, qn)):
        assert np.abs(want - base).max() > 1e-8
        assert np.abs(got - want).max() <= 1e-4 * np.abs(want - base).max(), np.abs(got - want).max()
    s.close()
