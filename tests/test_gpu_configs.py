"""The GPU path against stored oracle results on the larger workloads.

- a 150 x 20 sub-box of the 4096 x 20 generator (3000 beads, phi 0.20, xi 0.348);
- 8 of the 64 uneven systems of the batched form (254 - 1956 beads, phi 0.02 - 0.22,
  xi = 25/L), alone and solved together in one batch;
- one Brownian serving request (804 beads in aggregates of 29, phi 0.22, shear rate 1 on
  the sheared lattice, kT = 1, dt = 1e-3), given its real-space and near-field noise
  (grid noise zero), splitting parameter 25/L.

The oracle results come from tests/golden/make_golden.py, which calls only the oracle.
Parity runs tighten the Ewald and solver tolerances (1e-6 and 1e-7) so that the method's
own truncation and iteration errors stay well below the 1e-5 bar on the aggregate
velocities (translational and rotational parts separately); runs at each workload's own
tolerance (1e-5 for both) are held to 1e-4 and their errors are printed.
"""
import os

import numpy as np
import pytest

import fsdgen
from tests.golden.make_golden import REQUEST_NOISE_SEED, REQUEST_PICK, UNEVEN_PICK, digest

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PARITY = dict(ewald_tol=1e-6, gmres_tol=1e-7, gmres_maxit=5000)


@pytest.fixture(scope="module")
def F(gpu):
    import paper_2607_25161_amd as F
    return F


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_golden.py)")
    return np.load(path, allow_pickle=False)


def _errors(U, Uo):
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return rel(U[:, :3], Uo[:, :3]), rel(U[:, 3:], Uo[:, 3:])


@pytest.fixture(scope="module")
def c3sub():
    return fsdgen.config(2, n_agg=150, grid=0, name="clusters-150x20")


@pytest.mark.parametrize("precision", [0, 1])
def test_c3_subbox_matches_oracle(F, c3sub, precision):
    g = _golden("clusters150x20_oracle.npz")
    assert str(g["digest"]) == digest(c3sub)
    print(f"\n[c3sub] {c3sub.n_bead} beads, precision {precision}", flush=True)
    s = F.System.from_suspension(c3sub, precision=precision, **PARITY)
    U, _, info = s.solve()
    et, er = _errors(U, g["U"])
    print(f"  parity run: grid {s.info().grid}, xi {s.info().xi}, its {info.iterations}, err {et:.2e} {er:.2e}")
    assert info.rel_residual_fp64 <= 1e-7
    assert et < 1e-5 and er < 1e-5, (et, er)
    s.close()
    s = F.System.from_suspension(c3sub, precision=precision)   # the workload's own tolerance 1e-5
    U, _, info = s.solve()
    et, er = _errors(U, g["U"])
    print(f"  at tol 1e-5: support {s.info().support}, its {info.iterations}, err {et:.2e} {er:.2e}")
    assert info.rel_residual_fp64 <= 1e-5
    assert et < 1e-4 and er < 1e-4, (et, er)
    s.close()


@pytest.fixture(scope="module")
def uneven8():
    return [fsdgen.uneven_system(k) for k in UNEVEN_PICK]


@pytest.mark.parametrize("precision", [0, 1])
def test_uneven_systems_match_oracle(F, uneven8, precision):
    g = _golden("uneven8_oracle.npz")
    assert tuple(int(k) for k in g["picks"]) == UNEVEN_PICK
    for k, s0 in zip(UNEVEN_PICK, uneven8):
        assert str(g[f"digest_{k}"]) == digest(s0)
        print(f"\n[uneven {k}] {s0.n_bead} beads, precision {precision}", flush=True)
        s = F.System.from_suspension(s0, precision=precision, **PARITY)
        U, _, info = s.solve()
        et, er = _errors(U, g[f"U_{k}"])
        print(f"  parity run: grid {s.info().grid}, its {info.iterations}, err {et:.2e} {er:.2e}")
        assert et < 1e-5 and er < 1e-5, (k, et, er)
        s.close()
        s = F.System.from_suspension(s0, precision=precision)
        U, _, info = s.solve()
        et, er = _errors(U, g[f"U_{k}"])
        print(f"  at tol 1e-5: its {info.iterations}, err {et:.2e} {er:.2e}")
        assert info.rel_residual_fp64 <= 1e-5
        assert et < 1e-4 and er < 1e-4, (k, et, er)
        s.close()


@pytest.mark.parametrize("fused", [True, False])
def test_uneven_systems_in_one_batch_match_oracle(F, uneven8, fused):
    """The 8 systems solved together (mixed precision), with multi-system launches or one
    stream per system, each against its own oracle result."""
    g = _golden("uneven8_oracle.npz")
    systems = [F.System.from_suspension(s0, precision=F.FSD_MIXED, **PARITY) for s0 in uneven8]
    b = F.Batch(1 << 40, len(systems))
    b.set_fused(fused)
    slots = [b.admit(s) for s in systems]
    print(f"\n[batch fused={fused}] {sum(s.n_bead for s in uneven8)} beads", flush=True)
    assert b.solve() == 0
    for k, s, sl in zip(UNEVEN_PICK, systems, slots):
        info = b.info(sl)
        U = s.velocities()
        et, er = _errors(U, g[f"U_{k}"])
        print(f"  system {k}: its {info.iterations}, err {et:.2e} {er:.2e}")
        assert info.status == 0 and info.rel_residual_fp64 <= 1e-7
        assert et < 1e-5 and er < 1e-5, (k, et, er)
    b.close()
    for s in systems:
        s.close()


def test_brownian_request_matches_oracle(F):
    g = _golden("request27_oracle.npz")
    s0 = fsdgen.serving_request(REQUEST_PICK, kT=1.0, shear_rate=1.0)
    assert str(g["digest"]) == digest(s0)
    xi = float(g["xi"])
    assert xi == 25.0 / s0.L
    psi_r, psi_nf = fsdgen.brownian_noise(s0.n_bead, REQUEST_NOISE_SEED)
    print(f"\n[request {REQUEST_PICK}] {s0.n_bead} beads, sheared lattice", flush=True)
    k = int(g["lanczos_steps"])
    # the near-field root takes exactly k Lanczos steps (the tolerance is below what k steps
    # reach on the singular lubrication matrix); the real-space root converges well before k
    s = F.System.from_suspension(s0, lees_edwards=True, xi=xi, lanczos_tol=1e-10, lanczos_maxit=k, **PARITY)
    s.set_brownian(s0.dt)
    grid = s.info().grid
    s.set_noise(psi_w=np.zeros(3 * grid ** 3), psi_r=psi_r, psi_nf=psi_nf)
    _, _, steps = s.brownian_terms()
    assert steps[1] == k and steps[0] < k, steps
    U, _, info = s.solve()
    et, er = _errors(U, g["U"])
    print(f"  grid {grid}, its {info.iterations}, lanczos {steps}, err {et:.2e} {er:.2e}")
    assert info.rel_residual_fp64 <= 1e-7
    assert et < 1e-5 and er < 1e-5, (et, er)
    s.close()
