"""The continuous-batching server on the GPU: a request served in a mix of
others ends exactly where it ends when served alone, and its trajectory matches
the CPU oracle's."""
import numpy as np
import pytest

import fsdgen
from oracle import integrate, saddle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F(gpu):
    import paper_2607_25161_amd as F
    return F


def _requests(n, n_steps):
    return fsdgen.serving_requests(n, seed=fsdgen.BASE_SEED + 50, n_range=(60, 500), n_steps=n_steps)


@pytest.mark.parametrize("precision", [0, 1])
def test_request_in_mix_equals_alone(F, precision):
    from paper_2607_25161_amd.serving import BatchEngine, LibBackend, Request
    n_steps = 3
    reqs = _requests(5, n_steps)
    alone = []
    for s0 in reqs:
        s = F.System.from_suspension(s0, precision=precision)
        info = s.step(1e-3, n_steps)
        assert info.status == 0
        alone.append(s.state())
        s.close()
    be = LibBackend(F, 1 << 34, 2, dict(precision=precision))
    eng = BatchEngine(be, max_slots=2, dt=1e-3)
    # staggered request lengths so that slots turn over mid-run
    rs = [Request(k, s0, n_steps + (k % 2), arrival=0.0) for k, s0 in enumerate(reqs)]
    rep = eng.run(rs)
    assert rep["completed"] == 5 and rep["failed"] == 0
    assert eng.ticks > max(r.n_steps for r in rs)          # requests overlapped but not all at once
    for r in eng.done:
        X, q = r.result
        if r.n_steps == n_steps:
            Xa, qa = alone[r.rid]
            s0 = r.suspension
            if precision == 0:
                tx, tq = 1e-12 * s0.L, 1e-12
            else:
                # FP32 matvecs summed in another order by the multi-system launches: the
                # two runs agree to the solver tolerance (1e-5), 10x margin on the motion
                L = s0.L
                dX = np.abs((Xa - s0.com + L / 2) % L - L / 2).max()
                tx, tq = 1e-4 * dX + 1e-12 * L, 1e-4 * np.abs(qa - s0.quat).max() + 1e-12
            assert np.abs(X - Xa).max() <= tx, r.rid
            assert np.abs(q - qa).max() <= tq, r.rid
    be.batch.close()


def test_served_trajectory_matches_oracle(F):
    from paper_2607_25161_amd.serving import BatchEngine, LibBackend, Request
    n_steps, dt = 2, 1e-3
    s0 = _requests(1, n_steps)[0]
    s0.ewald_tol = s0.gmres_tol = 1e-8
    be = LibBackend(F, 1 << 34, 1, {})
    eng = BatchEngine(be, max_slots=1, dt=dt)
    eng.run([Request(0, s0, n_steps)])
    X, q = eng.done[0].result
    # oracle: the same explicit Euler steps with dense FP64 solves
    X0 = s0.com.copy()
    com, quat = s0.com.copy(), s0.quat.copy()
    for _ in range(n_steps):
        s0.com, s0.quat = com, quat
        U, *_ = saddle.solve_suspension(s0)
        com, quat = integrate.euler_step(com, quat, U, dt, s0.L)
    L = s0.L
    dX = (X - X0 + L / 2) % L - L / 2       # total displacement, minimum image
    dXo = (com - X0 + L / 2) % L - L / 2
    assert np.linalg.norm(dX - dXo) <= 1e-5 * np.linalg.norm(dXo)
    assert np.abs(q - quat).max() <= 1e-5 * dt
    be.batch.close()


def test_sheared_requests_in_mix_equal_alone(F):
    """Requests on the sheared lattice (shear rate 1, Brownian) served in a mix: each result
    equals the same request stepped alone, strain included."""
    from paper_2607_25161_amd.serving import BatchEngine, LibBackend, Request
    reqs = fsdgen.serving_requests(3, seed=91, n_range=(100, 400), n_steps=3, kT=1.0, shear_rate=1.0)
    be = LibBackend(F, 1 << 34, 3, {}, lees_edwards=True)
    eng = BatchEngine(be, max_slots=3, dt=1e-3)
    rep = eng.run([Request(k, s, 3) for k, s in enumerate(reqs)])
    assert rep["completed"] == 3 and rep["failed"] == 0
    served = {r.rid: r.result for r in eng.done}
    for k, s in enumerate(reqs):
        alone = F.System.from_suspension(s, lees_edwards=True)
        for _ in range(3):
            assert alone.step(1e-3, 1).status == 0
        X, q = alone.state()
        Xm, qm = served[k]
        assert np.abs(X - Xm).max() < 1e-9 and np.abs(q - qm).max() < 1e-9, k
        assert abs(alone.strain() - 3e-3) < 1e-15
        alone.close()
    be.batch.close()


@pytest.mark.parametrize("drift", [1, 2])
def test_brownian_requests_with_drift_in_mix_equal_alone(F, drift):
    """Brownian requests served with the drift on (random finite differences, Fixman): each
    result equals the same request stepped alone with that drift."""
    from paper_2607_25161_amd.serving import BatchEngine, LibBackend, Request
    reqs = fsdgen.serving_requests(3, seed=93, n_range=(100, 400), n_steps=2, kT=1.0)
    be = LibBackend(F, 1 << 34, 3, {}, drift=drift)
    eng = BatchEngine(be, max_slots=3, dt=1e-3)
    rep = eng.run([Request(k, s, 2) for k, s in enumerate(reqs)])
    assert rep["completed"] == 3 and rep["failed"] == 0
    served = {r.rid: r.result for r in eng.done}
    for k, s in enumerate(reqs):
        alone = F.System.from_suspension(s)
        alone.set_drift(drift)
        for _ in range(2):
            assert alone.step(1e-3, 1).status == 0
        X, q = alone.state()
        Xm, qm = served[k]
        assert np.abs(X - Xm).max() < 1e-9 and np.abs(q - qm).max() < 1e-9, k
        alone.close()
    be.batch.close()
