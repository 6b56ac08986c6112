"""Brownian terms on the GPU (Eq. `SP2`, Algorithm 1 step 3) through the C ABI.

- the device Philox4x64-10 generator against numpy's independent implementation;
- the wave-space square root: B B^T over all unit grid noises equals the wave-space
  mobility the library applies;
- the Lanczos real-space and near-field square roots against the oracle's exact
  square roots for the same noise;
- a full Brownian solve against the oracle given the same noise;
- the sample covariance of generated slip velocities against 2 kT / dt M.
"""
import math

import numpy as np
import pytest

import fsdgen
from oracle import brownian, rigid, saddle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F(gpu):
    import paper_2607_25161_amd as F
    return F


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _system(seed=21, sizes=(3, 4, 1, 5, 2), L=11.0, lub_on=True):
    rng = fsdgen.rng_from(seed)
    shapes = [fsdgen.sticking_cluster(rng, nb) for nb in sizes]
    com, quat = fsdgen.place_clusters(rng, shapes, L, gap=0.05)
    offs = np.r_[0, np.cumsum([len(s) for s in shapes])].astype(np.int32)
    return dict(L=L, a=1.0, eta=1.0, offsets=offs, x_body=np.concatenate(shapes), com=com, quat=quat,
                force=rng.normal(size=(len(sizes), 6)), grad_u=fsdgen.simple_shear(1.0),
                r_lub=3.0 if lub_on else 0.0)


def _make(F, kw, **p):
    par = dict(xi=0.6, ewald_tol=1e-10, r_lub=kw["r_lub"], r_precond=2.1 if kw["r_lub"] else 0.0,
               gmres_tol=1e-11, gmres_restart=40, gmres_maxit=3000, kT=0.5, lanczos_tol=1e-12)
    par.update(p)
    s = F.System(F.default_params(**par))
    s.init_box(kw["L"])
    s.init_aggregates(kw["offsets"], kw["x_body"], kw["com"], kw["quat"])
    s.set_forces(kw["force"])
    s.set_shear(kw["grad_u"])
    s.set_brownian(1.0)  # dt = 1, so the amplitude sqrt(2 kT / dt) is 1
    return s


def test_philox_matches_numpy(F):
    key = (0x243F6A8885A308D3, 0x13198A2E03707344)
    out = F.philox4x64(key[0], key[1], [5, 7, 9, 11], 64)
    # numpy's Philox advances its counter before each block: start one below
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array([4, 7, 9, 11], dtype=np.uint64))
    assert np.array_equal(out, bg.random_raw(256))


def test_normals_follow_box_muller_of_the_stream(F):
    k0, k1, purpose, step = 2607251610, 3, 1, 17
    z = F.normals(k0, k1, purpose, step, 4096)
    raw = np.random.Philox(key=np.array([k0, k1], dtype=np.uint64),
                           counter=np.array([0, purpose, step, 0], dtype=np.uint64)).random_raw(4096)
    u = ((raw >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    ref = np.empty(4096)
    ref[0::2] = r * np.cos(2 * np.pi * u2)
    ref[1::2] = r * np.sin(2 * np.pi * u2)
    assert np.abs(z - ref).max() < 1e-13
    big = F.normals(k0, k1, 0, 0, 1 << 20)
    n = big.size
    assert abs(big.mean()) < 5 / math.sqrt(n)
    assert abs(big.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(np.mean(big ** 4) - 3) < 5 * math.sqrt(96 / n)


def test_wave_square_root_reproduces_wave_mobility(F):
    """sum over unit grid noises e_m of (B e_m)(B e_m)^T = M_w, exactly up to rounding."""
    kw = _system(sizes=(2, 1, 3), L=9.0, lub_on=False)
    s = _make(F, kw, xi=0.4, ewald_tol=1e-3, grid=8)
    info = s.info()
    N, nb = info.grid, s.n_bead
    assert N == 8
    zr = np.zeros(6 * nb)
    cols = []
    e = np.zeros(3 * N ** 3)
    for m in range(3 * N ** 3):
        e[:] = 0
        e[m] = 1.0
        s.set_noise(psi_w=e, psi_r=zr)
        u, f, its = s.brownian_terms()
        cols.append(u.ravel())
    B = np.array(cols).T
    Mw = np.column_stack([s.apply_mobility(c, parts=2) for c in np.eye(6 * nb)])
    assert np.abs(B @ B.T - Mw).max() <= 1e-12 * np.abs(Mw).max()


def test_real_space_square_root_matches_oracle(F):
    kw = _system(lub_on=False)
    s = _make(F, kw)
    info = s.info()
    nb = s.n_bead
    rng = np.random.default_rng(12)
    psi_r = rng.normal(size=6 * nb)
    s.set_noise(psi_w=np.zeros(3 * info.grid ** 3), psi_r=psi_r)
    u, f, its = s.brownian_terms()
    A = saddle.assemble(**kw)
    ref = brownian.real_space_slip(A.x, kw["L"], 1.0, 1.0, info.xi, info.r_cut, psi_r, 0.5, 1.0)
    assert _rel(u, ref) < 1e-8, its
    assert np.all(f == 0) and 0 < its[0] < 100


def test_near_field_square_root_matches_oracle(F):
    kw = _system(seed=23, sizes=(4, 4, 3, 5, 2, 6), L=10.0)
    s = _make(F, kw)
    info = s.info()
    nb = s.n_bead
    assert info.n_lub_pairs > 0
    rng = np.random.default_rng(13)
    psi_nf = rng.normal(size=3 * nb)
    s.set_noise(psi_w=np.zeros(3 * info.grid ** 3), psi_r=np.zeros(6 * nb), psi_nf=psi_nf)
    u, f, its = s.brownian_terms()
    A = saddle.assemble(**kw)
    body = rigid.body_index(kw["offsets"])
    ref = brownian.near_field_force(A.x, body, kw["L"], 1.0, 1.0, 3.0, psi_nf, 0.5, 1.0)
    # R_nf is singular (rigid translations of connected pairs, every rotation); the square
    # root of eigenvalues that rounding leaves at +-1e-15 of the largest is ~3e-8 of it, so
    # both the exact root and the Lanczos root carry ~1e-8 in those components
    assert _rel(f, ref) < 1e-7, (_rel(f, ref), its)
    assert np.abs(u).max() == 0


def test_brownian_solve_matches_oracle(F):
    """Full solve with explicit real-space and near-field noise (grid noise zero)."""
    kw = _system(seed=24, sizes=(4, 4, 3, 5, 2, 6), L=10.0)
    s = _make(F, kw, kT=0.8)
    s.set_brownian(0.01)
    info = s.info()
    nb = s.n_bead
    rng = np.random.default_rng(14)
    psi_r, psi_nf = rng.normal(size=6 * nb), rng.normal(size=3 * nb)
    s.set_noise(psi_w=np.zeros(3 * info.grid ** 3), psi_r=psi_r, psi_nf=psi_nf)
    U, _, sinfo = s.solve()
    A = saddle.assemble(**kw)
    body = rigid.body_index(kw["offsets"])
    ub = brownian.real_space_slip(A.x, kw["L"], 1.0, 1.0, info.xi, info.r_cut, psi_r, 0.8, 0.01)
    fb3 = brownian.near_field_force(A.x, body, kw["L"], 1.0, 1.0, 3.0, psi_nf, 0.8, 0.01)
    fb = np.zeros((nb, 6))
    fb[:, :3] = fb3
    Uo, *_ = saddle.solve(**kw, u_brown=ub, f_brown_nf=fb)
    assert _rel(U[:, :3], Uo[:, :3]) < 1e-7 and _rel(U[:, 3:], Uo[:, 3:]) < 1e-7


def test_generated_slip_covariance(F):
    """<u_B u_B^T> -> (2 kT/dt) (M_r + M_w) for generated noise (statistical, 3 beads)."""
    kw = _system(seed=25, sizes=(1, 1, 1), L=8.0, lub_on=False)
    s = _make(F, kw, ewald_tol=1e-6, lanczos_tol=1e-8)
    nb = s.n_bead
    K = 10000
    U = np.empty((K, 6 * nb))
    for k in range(K):
        s.set_brownian(1.0, step=k)
        u, f, its = s.brownian_terms()
        U[k] = u.ravel()
    C = U.T @ U / K
    M = np.column_stack([s.apply_mobility(c) for c in np.eye(6 * nb)])
    target = 2 * 0.5 / 1.0 * M
    # sample covariance of K Gaussian vectors: E|C - S|_F^2 = (tr(S)^2 + |S|_F^2) / K, so the
    # relative error is at most sqrt(19 / K) = 0.044 in RMS for these 18 dimensions
    assert np.linalg.norm(C - target) <= 0.12 * np.linalg.norm(target)
    assert abs(U.mean()) < 0.05 * math.sqrt(np.abs(np.diag(target)).max())


def test_brownian_steps_reproducible_by_seed(F):
    kw = _system(seed=26)
    runs = []
    for seed in (1, 1, 2):
        s = _make(F, kw, kT=1.0, seed=seed, gmres_tol=1e-8, lanczos_tol=1e-4, ewald_tol=1e-6)
        s.step(1e-3, 3)
        runs.append(s.state())
        s.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    assert np.abs(runs[0][0] - runs[2][0]).max() > 1e-6
