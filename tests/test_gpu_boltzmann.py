"""Two-particle Boltzmann check of the Brownian drift (Appendix A, both estimators).

Pairs of single-bead bodies are held near the separation r0 = 3a by the linear potential
V(r) = k_n |r - r0| with k_n = 3 kT (the appendix prints the potential with a minus
sign, which has no equilibrium; the well is the reading taken), with lubrication on
and contact kept by a stiff Hertz force.  Stepping with the drift of random finite
differences or of Fixman's midpoint scheme, the centre distance r of a pair must sample
the Boltzmann density P(r) ~ r^2 exp(-(V(r) + V_Hertz(r)) / kT).  The equilibrium density
does not depend on the mobility, so many pairs share one dilute periodic box (their
hydrodynamic coupling changes how fast they sample, not what): 32 pairs give 32 nearly
independent time series.  The test compares the sampled mean and variance of r with that
density, with error bars from the spread of the per-pair averages.
"""
import math
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KT, KN, R0, A = 1.0, 3.0, 3.0, 1.0
K_HERTZ = 1e3
NX, NY, NZ, SPACING = 4, 4, 2, 12.0  # pairs on a lattice, 12a apart (x, y) and 24a (z)
L = NX * SPACING
DT, STEPS, BURN = 0.02, 6000, 1000


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_25161_amd as F
    return F


def _density_moments():
    """Mean and variance of r under r^2 exp(-(V + V_Hertz)/kT) on a fine grid."""
    r = np.linspace(1.8, 12.0, 400001)
    v = KN * np.abs(r - R0) + np.where(r < 2 * A, 0.4 * K_HERTZ * np.clip(2 * A - r, 0, None) ** 2.5, 0.0)
    w = r ** 2 * np.exp(-v / KT)
    w /= np.trapezoid(w, r)
    m = np.trapezoid(w * r, r)
    return m, np.trapezoid(w * (r - m) ** 2, r)


def _run(F, mode, seed):
    npair = NX * NY * NZ
    centres = np.array([[(i + 0.5) * SPACING, (j + 0.5) * SPACING, (k + 0.5) * 2 * SPACING]
                        for i in range(NX) for j in range(NY) for k in range(NZ)]) - L / 2
    com = np.empty((2 * npair, 3))
    com[0::2] = centres - [R0 / 2, 0, 0]
    com[1::2] = centres + [R0 / 2, 0, 0]
    s = F.System(eta=1.0, radius=A, kT=KT, xi=0.0, ewald_tol=1e-4, gmres_tol=1e-6, seed=seed)
    s.init_box(L)
    s.init_aggregates(np.arange(2 * npair + 1), np.zeros((2 * npair, 3)), com,
                      np.tile([1.0, 0, 0, 0], (2 * npair, 1)))
    s.set_pair_forces(k_n=K_HERTZ, r_cut=2.0 * A)
    s.set_warm_start(1)
    if mode:
        s.set_drift(mode)
    rs = np.empty((STEPS - BURN, npair))
    ft = np.zeros((2 * npair, 6))
    t0 = time.perf_counter()
    for k in range(STEPS):
        X, _ = s.state()
        d = X[0::2] - X[1::2]
        d -= L * np.round(d / L)
        r = np.linalg.norm(d, axis=1)
        f = -KN * np.sign(r - R0)[:, None] * d / r[:, None]
        ft[0::2, :3] = f
        ft[1::2, :3] = -f
        s.set_forces(ft)
        info = s.step(DT, 1)
        assert info.status == 0, (mode, k, info.status)
        if k >= BURN:
            rs[k - BURN] = r
    el = time.perf_counter() - t0
    s.close()
    # per-pair averages are close to independent: their spread sets the error bars
    means, var2 = rs.mean(axis=0), ((rs - rs.mean()) ** 2).mean(axis=0)
    return rs.ravel(), means.std(ddof=1) / math.sqrt(npair), var2.std(ddof=1) / math.sqrt(npair), el


@pytest.mark.parametrize("mode,name", [(1, "random finite differences"), (2, "Fixman")])
def test_drift_samples_boltzmann_distance(F, mode, name):
    m_th, v_th = _density_moments()
    rs, se_m, se_v, el = _run(F, mode, seed=101 + mode)
    hist, edges = np.histogram(rs, bins=np.linspace(1.9, 5.5, 19), density=True)
    print(f"\n[{name}] {NX * NY * NZ} pairs, {STEPS} steps of dt {DT} in {el:.1f} s: mean r {rs.mean():.4f} "
          f"+- {se_m:.4f} "
          f"(Boltzmann {m_th:.4f}), var {rs.var():.4f} +- {se_v:.4f} (Boltzmann {v_th:.4f})", flush=True)
    print("  P(r) by bin:", " ".join(f"{h:.3f}" for h in hist), flush=True)
    # 4 standard errors plus an allowance for the O(dt) bias of the Euler-Maruyama step
    assert abs(rs.mean() - m_th) < 4 * se_m + 0.01, (rs.mean(), m_th, se_m)
    assert abs(rs.var() - v_th) < 4 * se_v + 0.01, (rs.var(), v_th, se_v)
