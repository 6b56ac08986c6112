"""Seeded synthetic suspensions of rigid bead aggregates.

This module only *draws inputs*: aggregate shapes, their placement in a periodic
cube, orientations and the imposed forcing.  It holds none of the arithmetic of
the solve (no mobility, no constraint matrices, no quaternion kinematics of the
integrator).  Both the CPU oracle and the GPU path consume what it returns.

Shapes follow the random-sticking growth rule of the paper's carbon-black
generator (Section 4.1, Eq. `prob`): the next bead touches an existing bead
chosen with probability P(d_i) = 1 - (1 - d_i) k_p, where d_i is the bead's
normalised distance sum.  For k_p > 1 that expression goes negative near the
cluster core; it is clamped at zero.

Placement is random sequential addition in a cube of side
L = (N_tot (4 pi / 3) a^3 / phi)^(1/3), with uniform random orientations
(Shoemake's method) and a minimum inter-body surface gap.  Above a packing
that RSA cannot reach, cluster centres fall back to a jittered lattice.

All randomness comes from numpy's Philox counter-based generator keyed by the
seed, so every workload is reproducible from (config, seed).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
from scipy.spatial.transform import Rotation

BASE_SEED = 2607251610


def rng_from(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed) & ((1 << 64) - 1)))


# --------------------------------------------------------------------------
# shapes
# --------------------------------------------------------------------------

def doublet(a: float = 1.0) -> np.ndarray:
    """Two touching beads along the body x axis, centroid at the origin."""
    return np.array([[-a, 0.0, 0.0], [a, 0.0, 0.0]])


def _unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def sticking_cluster(rng, n_b: int, a: float = 1.0, k_p: float = 2.0,
                     max_tries: int = 400) -> np.ndarray:
    """Random-sticking aggregate of n_b touching beads (centre distance 2a).

    A candidate bead is rejected if it comes closer than 2a to any bead other
    than the one it attaches to.  The returned coordinates are relative to the
    bead centroid.
    """
    if n_b < 1:
        raise ValueError("n_b must be >= 1")
    x = np.zeros((n_b, 3))
    if n_b == 1:
        return x
    x[1] = 2.0 * a * _unit_vectors(rng, 1)[0]
    for m in range(2, n_b):
        placed = False
        for _ in range(max_tries):
            cur = x[:m]
            dsum = np.linalg.norm(cur[:, None, :] - cur[None, :, :], axis=2).sum(1)
            d = dsum / dsum.max()
            p = np.clip(1.0 - (1.0 - d) * k_p, 0.0, None)
            if p.sum() <= 0.0:
                p = np.ones(m)
            p = p / p.sum()
            i = rng.choice(m, p=p)
            cand = cur[i] + 2.0 * a * _unit_vectors(rng, 1)[0]
            dist = np.linalg.norm(cur - cand, axis=1)
            dist[i] = np.inf
            if np.all(dist >= 2.0 * a * (1.0 - 1e-12)):
                x[m] = cand
                placed = True
                break
        if not placed:
            raise RuntimeError("sticking_cluster: could not place bead")
    return x - x.mean(axis=0)


def uniform_quaternion(rng) -> np.ndarray:
    """Uniform random unit quaternion (w, x, y, z), Shoemake's subgroup method."""
    u1, u2, u3 = rng.random(3)
    s1, s2 = math.sqrt(1.0 - u1), math.sqrt(u1)
    t1, t2 = 2.0 * math.pi * u2, 2.0 * math.pi * u3
    q = np.array([s2 * math.cos(t2), s1 * math.sin(t1), s1 * math.cos(t1), s2 * math.sin(t2)])
    if q[0] < 0:
        q = -q
    return q


def _rotate(q_wxyz, pts):
    # scipy uses scalar-last quaternions; only used to check overlaps here.
    return Rotation.from_quat([q_wxyz[1], q_wxyz[2], q_wxyz[3], q_wxyz[0]]).apply(pts)


# --------------------------------------------------------------------------
# placement
# --------------------------------------------------------------------------

class _CellGrid:
    """Bucket grid over the periodic box used for overlap checks while placing."""

    def __init__(self, L, cell):
        self.L = L
        self.nc = max(1, int(L // cell))
        self.cell = L / self.nc
        self.buckets: dict = {}

    def _key(self, p):
        c = np.floor((p % self.L) / self.cell).astype(int) % self.nc
        return int(c[0]), int(c[1]), int(c[2])

    def near(self, p):
        cx, cy, cz = self._key(p)
        out = []
        rng = (-1, 0, 1) if self.nc >= 3 else range(self.nc)
        seen = set()
        for dx in rng:
            for dy in rng:
                for dz in rng:
                    k = ((cx + dx) % self.nc, (cy + dy) % self.nc, (cz + dz) % self.nc)
                    if k in seen:
                        continue
                    seen.add(k)
                    out.extend(self.buckets.get(k, ()))
        return out

    def add(self, p, payload):
        self.buckets.setdefault(self._key(p), []).append(payload)


def _fits(grid, pts, L, min_dist, placed_pos):
    for p in pts:
        idx = grid.near(p)
        if not idx:
            continue
        q = placed_pos[idx]
        d = q - p
        d -= L * np.round(d / L)
        if np.any(np.einsum("ij,ij->i", d, d) < min_dist * min_dist):
            return False
    return True


def place_clusters(rng, shapes, L, a=1.0, gap=0.01, max_tries=2000):
    """Random sequential addition of rigid clusters in a periodic cube.

    Returns (com, quat) with com in [-L/2, L/2)^3 and quat (w,x,y,z).  A
    placement is accepted when every inter-body bead pair is at least 2a + gap
    apart (minimum image).  Clusters that RSA cannot place go on a jittered
    lattice of candidate centres tried in random order.
    """
    n = len(shapes)
    cell = 2.0 * a + gap
    grid = _CellGrid(L, cell)
    placed_pos = np.zeros((sum(len(s) for s in shapes), 3))
    n_placed = 0
    com = np.zeros((n, 3))
    quat = np.zeros((n, 4))
    order = np.argsort([-len(s) for s in shapes], kind="stable")
    lattice = None
    for c in order:
        shape = shapes[c]
        ok = False
        for t in range(max_tries):
            if t < max_tries // 2 or lattice is None:
                X = (rng.random(3) - 0.5) * L
            else:
                X = lattice[rng.integers(len(lattice))] + (rng.random(3) - 0.5) * 0.2 * a
            q = uniform_quaternion(rng)
            pts = X + _rotate(q, shape)
            if _fits(grid, pts, L, 2.0 * a + gap, placed_pos):
                ok = True
                break
            if t == max_tries // 2 and lattice is None:
                m = int(math.ceil(n ** (1.0 / 3.0))) + 1
                g = (np.arange(m) + 0.5) / m * L - L / 2
                lattice = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
        if not ok:
            raise RuntimeError("place_clusters: packing too dense for RSA")
        com[c] = X
        quat[c] = q
        for p in pts:
            placed_pos[n_placed] = p
            grid.add(p, n_placed)
            n_placed += 1
    com = (com + L / 2) % L - L / 2
    return com, quat


def grow_in_box(rng, sizes, L, a=1.0, gap=0.01, k_p=2.0, max_tries=200):
    """Grow random-sticking clusters directly inside the periodic box.

    For dense suspensions, where rigid clusters cannot be inserted at random,
    each cluster starts from a free seed position and grows bead by bead with the
    sticking rule of `sticking_cluster`; a candidate bead must keep 2a from its own
    cluster (except the bead it touches) and 2a + gap from every other body
    (minimum image).  Each finished cluster gets a uniform random orientation: its
    body-frame coordinates are the lab offsets from the centroid rotated back by
    that orientation.  Returns (shapes, com, quat).
    """
    grid = _CellGrid(L, 2.0 * a + gap)
    placed = np.zeros((sum(sizes), 3))
    n_placed = 0
    shapes, coms, quats = [], [], []
    for nb in sizes:
        for _restart in range(50):
            own = []
            for _ in range(max_tries):
                X0 = (rng.random(3) - 0.5) * L
                if _fits(grid, [X0], L, 2.0 * a + gap, placed):
                    own.append(X0)
                    break
            if not own:
                continue
            ok = True
            for m in range(1, nb):
                cur = np.array(own)
                done = False
                for _ in range(max_tries):
                    if m == 1:
                        i = 0
                    else:
                        dsum = np.linalg.norm(cur[:, None, :] - cur[None, :, :], axis=2).sum(1)
                        d = dsum / dsum.max()
                        pr = np.clip(1.0 - (1.0 - d) * k_p, 0.0, None)
                        pr = pr / pr.sum() if pr.sum() > 0 else np.full(m, 1.0 / m)
                        i = rng.choice(m, p=pr)
                    cand = cur[i] + 2.0 * a * _unit_vectors(rng, 1)[0]
                    dist = np.linalg.norm(cur - cand, axis=1)
                    dist[i] = np.inf
                    if np.all(dist >= 2.0 * a * (1.0 - 1e-12)) and _fits(grid, [cand], L, 2.0 * a + gap, placed):
                        own.append(cand)
                        done = True
                        break
                if not done:
                    ok = False
                    break
            if ok:
                break
        else:
            raise RuntimeError("grow_in_box: could not grow a cluster")
        pts = np.array(own)
        c = pts.mean(axis=0)
        q = uniform_quaternion(rng)
        body = Rotation.from_quat([q[1], q[2], q[3], q[0]]).inv().apply(pts - c)
        for p_ in pts:
            placed[n_placed] = p_
            grid.add(p_, n_placed)
            n_placed += 1
        shapes.append(body)
        coms.append(c)
        quats.append(q)
    com = (np.array(coms) + L / 2) % L - L / 2
    return shapes, com, np.array(quats)


def box_side(n_bead, phi, a=1.0):
    return (n_bead * (4.0 * math.pi / 3.0) * a ** 3 / phi) ** (1.0 / 3.0)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclass
class Suspension:
    """One periodic system: geometry, forcing and solver settings."""
    name: str
    L: float
    a: float
    eta: float
    offsets: np.ndarray          # (N+1,) int32, bead ranges per aggregate
    x_body: np.ndarray           # (Ntot, 3) bead vectors in the body frame, centroid 0
    com: np.ndarray              # (N, 3) centroids in [-L/2, L/2)^3
    quat: np.ndarray             # (N, 4) unit quaternions (w, x, y, z)
    force: np.ndarray            # (N, 6) applied force then torque per aggregate
    grad_u: np.ndarray           # (3, 3) imposed velocity gradient d u_a / d x_b
    xi: float                    # Ewald splitting parameter
    ewald_tol: float
    gmres_tol: float
    grid: int                    # 0: from the cutoff rule
    r_lub: float                 # 0 disables lubrication
    r_precond: float
    kT: float = 0.0
    dt: float = 1e-3
    n_steps: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def n_agg(self):
        return len(self.offsets) - 1

    @property
    def n_bead(self):
        return int(self.offsets[-1])

    @property
    def phi(self):
        return self.n_bead * (4 * math.pi / 3) * self.a ** 3 / self.L ** 3


def _assemble(name, shapes, L, rng, a=1.0, gap=0.01, **kw):
    com, quat = place_clusters(rng, shapes, L, a=a, gap=gap)
    offsets = np.zeros(len(shapes) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([len(s) for s in shapes])
    x_body = np.concatenate(shapes, axis=0)
    return dict(name=name, L=L, a=a, offsets=offsets, x_body=x_body, com=com, quat=quat)


def _dense_assemble(name, sizes, L, rng, a=1.0, gap=0.01, k_p=2.0):
    shapes, com, quat = grow_in_box(rng, sizes, L, a=a, gap=gap, k_p=k_p)
    offsets = np.zeros(len(shapes) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([len(s) for s in shapes])
    return dict(name=name, L=L, a=a, offsets=offsets, x_body=np.concatenate(shapes), com=com, quat=quat)


def simple_shear(rate=1.0):
    g = np.zeros((3, 3))
    g[0, 1] = rate          # u = rate * y * x_hat
    return g


def sedimenting_doublets(seed=BASE_SEED + 1, n_agg=16, phi=0.05, a=1.0):
    """16 touching doublets, unit force -z on each, no shear, no lubrication."""
    rng = rng_from(seed)
    shapes = [doublet(a) for _ in range(n_agg)]
    L = box_side(2 * n_agg, phi, a)
    g = _assemble("doublets-16", shapes, L, rng, a=a)
    force = np.zeros((n_agg, 6))
    force[:, 2] = -1.0
    return Suspension(eta=1.0, force=force, grad_u=np.zeros((3, 3)), xi=0.5 / a,
                      ewald_tol=1e-8, gmres_tol=1e-8, grid=0, r_lub=0.0, r_precond=0.0,
                      **g)


def sheared_clusters(seed=BASE_SEED + 2, n_agg=256, n_b=8, phi=0.10, a=1.0,
                     k_p=2.0, xi=0.5, tol=1e-6, grid=64, n_steps=10, name=None, dense=False):
    """Random-sticking clusters in simple shear with lubrication (cutoff 3a).

    dense=False grows each cluster alone and places it by random sequential
    addition; dense=True grows the clusters inside the box (for volume fractions
    that rigid insertion cannot reach).
    """
    rng = rng_from(seed)
    L = box_side(n_agg * n_b, phi, a)
    nm = name or f"clusters-{n_agg}x{n_b}"
    if dense:
        g = _dense_assemble(nm, [n_b] * n_agg, L, rng, a=a, k_p=k_p)
    else:
        shapes = [sticking_cluster(rng, n_b, a, k_p) for _ in range(n_agg)]
        g = _assemble(nm, shapes, L, rng, a=a)
    return Suspension(eta=1.0, force=np.zeros((n_agg, 6)), grad_u=simple_shear(1.0),
                      xi=xi / a, ewald_tol=tol, gmres_tol=tol, grid=grid,
                      r_lub=3.0 * a, r_precond=2.1 * a, n_steps=n_steps, **g)


def config(index: int, **overrides) -> Suspension:
    """Workloads by index: 0 doublets, 1 clusters 256x8, 2 clusters 4096x20."""
    if index == 0:
        return sedimenting_doublets(**overrides)
    if index == 1:
        return sheared_clusters(**overrides)
    if index == 2:
        kw = dict(seed=BASE_SEED + 3, n_agg=4096, n_b=20, phi=0.20, xi=0.348, tol=1e-5,
                  grid=128, n_steps=1, name="clusters-4096x20", dense=True)
        kw.update(overrides)
        return sheared_clusters(**kw)
    raise ValueError(index)


def uneven_system(k, seed=BASE_SEED + 4, n_range=(200, 4000), nb_range=(4, 30),
                  phi_range=(0.02, 0.25), tol=1e-5, a=1.0, k_p=2.0):
    """System k of the uneven set (its own seed, seed + k): bead count uniform in
    n_range, beads per aggregate uniform in nb_range (the last aggregate takes the
    remainder, at least 1 bead), volume fraction uniform in phi_range, splitting
    parameter 25 / L, simple shear and lubrication as in the sheared-cluster workload."""
    rng = rng_from(seed + k)
    n_tot = int(rng.integers(n_range[0], n_range[1] + 1))
    n_b = int(rng.integers(nb_range[0], nb_range[1] + 1))
    phi = float(rng.uniform(*phi_range))
    sizes = _split_sizes(n_tot, n_b)
    L = box_side(n_tot, phi, a)
    g = _dense_assemble(f"system-{k}", sizes, L, rng, a=a, k_p=k_p)
    return Suspension(eta=1.0, force=np.zeros((len(sizes), 6)), grad_u=simple_shear(1.0),
                      xi=25.0 / L, ewald_tol=tol, gmres_tol=tol, grid=0, r_lub=3.0 * a,
                      r_precond=2.1 * a, **g)


def uneven_systems(seed=BASE_SEED + 4, n_sys=64, **kw):
    """Independent periodic systems of uneven size for the batched form (`uneven_system`
    for k = 0 .. n_sys - 1)."""
    return [uneven_system(k, seed=seed, **kw) for k in range(n_sys)]


def _split_sizes(n_tot, n_b):
    sizes = [n_b] * (n_tot // n_b)
    if n_tot % n_b:
        sizes.append(n_tot % n_b)
    return sizes


def serving_request(r, seed=BASE_SEED + 5, n_range=(100, 50000), nb_range=(4, 30),
                    phi_range=(0.02, 0.25), tol=1e-5, n_steps=20, kT=0.0, a=1.0, k_p=2.0, maxit=20000,
                    shear_rate=0.01):
    """Request r of the serving stream, drawn from its own Philox stream keyed by
    (seed, r): bead count log-uniform in n_range, beads per aggregate uniform in
    nb_range, volume fraction uniform in phi_range; shear and lubrication as in the
    other workloads; splitting parameter and grid left to the library's policy
    (xi = 0, grid = 0); n_steps time steps.  Brownian motion (kT > 0) brings bodies
    into near contact, where the lubrication makes the saddle system stiff: the GMRES
    budget per solve is maxit.

    The shear rate is shear_rate.  On a cubic periodic box (no Lees-Edwards images)
    bodies facing each other across the y boundary move apart or together at
    shear_rate * L, and the default 0.01 keeps that relative motion over a request
    (shear_rate * L * n_steps * dt <= 0.05 a for L up to 220 a) below the smallest gaps
    the generator leaves; faster shear belongs on the sheared lattice, which removes
    that jump (the serving benchmark runs shear rate 1 there).
    """
    rng = np.random.Generator(np.random.Philox(key=np.uint64(seed & ((1 << 64) - 1)),
                                               counter=np.array([0, 0, 0, r], dtype=np.uint64)))
    n_tot = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
    n_b = int(rng.integers(nb_range[0], nb_range[1] + 1))
    phi = float(rng.uniform(*phi_range))
    sizes = _split_sizes(n_tot, n_b)
    L = box_side(n_tot, phi, a)
    g = _dense_assemble(f"request-{r}", sizes, L, rng, a=a, k_p=k_p)
    return Suspension(eta=1.0, force=np.zeros((len(sizes), 6)), grad_u=simple_shear(shear_rate),
                      xi=0.0, ewald_tol=tol, gmres_tol=tol, grid=0, r_lub=3.0 * a,
                      r_precond=2.1 * a, kT=kT, n_steps=n_steps, extra={"gmres_maxit": maxit}, **g)


def serving_requests(n_req, seed=BASE_SEED + 5, **kw):
    """A stream of independent simulation requests for the serving form
    (`serving_request` for r = 0 .. n_req - 1)."""
    return [serving_request(r, seed=seed, **kw) for r in range(n_req)]


def brownian_noise(n_bead, seed):
    """Standard normal inputs of one Brownian solve given from outside: psi_r (6 per bead,
    the real-space slip) and psi_nf (3 per bead, the near-field force)."""
    rng = rng_from(seed)
    return rng.normal(size=6 * n_bead), rng.normal(size=3 * n_bead)


def rod(n_b, a=1.0):
    """n_b touching beads on a straight line (centre spacing 2a) along x, centroid at 0."""
    x = (np.arange(n_b) - 0.5 * (n_b - 1)) * 2.0 * a
    return np.stack([x, np.zeros(n_b), np.zeros(n_b)], axis=1)


def _aligned_rods(rng, n_rod, n_b, L, a, gap):
    """Rods along x in columns on a square (y, z) lattice, as many per column as fit end to
    end, each column shifted along x at random (the fallback where isotropic placement fails)."""
    length = 2.0 * a * n_b
    per_col = int(L // (length + gap))
    n_col = -(-n_rod // per_col)
    m = int(math.ceil(math.sqrt(n_col)))
    if L / m < 2.0 * a + gap:
        raise RuntimeError("aligned rods do not fit either")
    com = np.zeros((n_rod, 3))
    k = 0
    for c in range(n_col):
        y, z = (c % m + 0.5) * L / m - L / 2, (c // m + 0.5) * L / m - L / 2
        x0 = rng.random() * L
        for r in range(per_col):
            if k == n_rod:
                break
            com[k] = [(x0 + r * L / per_col) % L - L / 2, y, z]
            k += 1
    offsets = np.arange(n_rod + 1, dtype=np.int32) * n_b
    quat = np.tile([1.0, 0.0, 0.0, 0.0], (n_rod, 1))
    return dict(name=f"rods-{n_rod}x{n_b}", L=L, a=a, offsets=offsets, x_body=np.tile(rod(n_b, a), (n_rod, 1)),
                com=com, quat=quat)


def brownian_rods(n_rod, n_b, phi, xi_policy="fixed", seed=BASE_SEED + 6, tol=1e-5, kT=1.0, dt=1e-3, a=1.0,
                  k_n=1e3):
    """Brownian rigid rods for the scaling study of Section 3.2: n_rod straight rods of n_b
    touching beads, uniformly random orientations and positions (random sequential addition,
    inter-body gaps of at least 0.1a) in a periodic cube at volume fraction phi, no imposed
    flow, thermal energy kT, Hertz contact between rods (stiffness k_n, in extra), lubrication
    as in the other workloads.  xi_policy "fixed" gives xi = 0.5/a, "box" gives xi = 25/L,
    the two policies of Section 3.2."""
    rng = rng_from(seed + 1000 * n_b + int(round(1000 * phi)))
    L = box_side(n_rod * n_b, phi, a)
    if 2.0 * a * n_b + 0.1 * a > L:
        raise ValueError("rods longer than the box would touch their own images")
    try:
        g = _assemble(f"rods-{n_rod}x{n_b}", [rod(n_b, a)] * n_rod, L, rng, a=a, gap=0.1 * a)
    except RuntimeError:  # long rods at this volume fraction: no isotropic packing by RSA
        g = _aligned_rods(rng, n_rod, n_b, L, a, 0.1 * a)
    xi = 0.5 / a if xi_policy == "fixed" else 25.0 / L
    return Suspension(eta=1.0, force=np.zeros((n_rod, 6)), grad_u=np.zeros((3, 3)), xi=xi, ewald_tol=tol,
                      gmres_tol=tol, grid=0, r_lub=3.0 * a, r_precond=2.1 * a, kT=kT, dt=dt,
                      extra={"k_n": k_n}, **g)


def random_force(rng, n_agg, scale=1.0):
    return scale * rng.normal(size=(n_agg, 6))
