"""Write oracle reference values for the full-size parity workloads.

Calls only the CPU oracle and the seeded generator.  Each output stores a
digest of the generated inputs so a test can confirm it regenerates the same
system before comparing.

    python tests/golden/make_golden.py doublets      # 16 doublets, one solve
    python tests/golden/make_golden.py clusters      # 256 x 8 clusters, 10 steps
    python tests/golden/make_golden.py c3sub         # 150 x 20 clusters of the 4096 x 20 generator
    python tests/golden/make_golden.py uneven        # 8 of the 64 uneven systems, one solve each
    python tests/golden/make_golden.py request       # one Brownian serving request, given noise
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fsdgen  # noqa: E402
from oracle import brownian, integrate, rigid, saddle  # noqa: E402

# systems of the 64-system uneven set with an oracle result (sizes 254 .. 1956 beads,
# volume fractions 0.02 .. 0.22, grids 64^3 .. 96^3 at xi = 25/L)
UNEVEN_PICK = (17, 3, 30, 41, 54, 28, 36, 62)
# the serving request with an oracle result: 804 beads in aggregates of 29, phi 0.22
REQUEST_PICK = 27
REQUEST_NOISE_SEED = fsdgen.BASE_SEED + 900
# Lanczos steps of the request's near-field root: its lubrication matrix is singular, so the
# Lanczos root is still 1e-3 away from the exact one after 100 steps and the stored value
# is the 100-step approximation itself
REQUEST_LANCZOS_STEPS = 100


def digest(s) -> str:
    h = hashlib.sha256()
    for arr in (s.offsets, s.x_body, s.com, s.quat, s.force, s.grad_u):
        h.update(np.ascontiguousarray(arr, dtype=np.float64).tobytes())
    h.update(np.float64([s.L, s.a, s.eta, s.r_lub]).tobytes())
    return h.hexdigest()


def run(index: int, n_steps: int, out: str):
    s = fsdgen.config(index)
    com, quat = s.com.copy(), s.quat.copy()
    Us, res = [], []
    for step in range(n_steps):
        t = time.time()
        U, F, r, A = saddle.solve(s.L, s.a, s.eta, s.offsets, s.x_body, com, quat, s.force,
                                  s.grad_u, r_lub=s.r_lub)
        Us.append(U)
        res.append(r)
        print(f"{s.name} step {step}: residual {r:.2e} ({time.time() - t:.1f} s)", flush=True)
        com, quat = integrate.euler_step(com, quat, U, s.dt, s.L)
    np.savez(os.path.join(HERE, out), digest=np.array(digest(s)), U=np.array(Us),
             residual=np.array(res), dt=s.dt, com_final=com, quat_final=quat)


def c3_sub():
    """One solve of a 150 x 20 sub-box of the 4096 x 20 generator (phi 0.20), at the
    oracle's own Ewald split (the result does not depend on it)."""
    s = fsdgen.config(2, n_agg=150, grid=0, name="clusters-150x20")
    t = time.time()
    U, F, r, A = saddle.solve_suspension(s)
    print(f"{s.name}: {s.n_bead} beads, residual {r:.2e} ({time.time() - t:.1f} s)", flush=True)
    np.savez(os.path.join(HERE, "clusters150x20_oracle.npz"), digest=np.array(digest(s)), U=U, residual=r)


def uneven():
    """One solve of each picked system of the uneven set."""
    out = {}
    for k in UNEVEN_PICK:
        s = fsdgen.uneven_system(k)
        t = time.time()
        U, F, r, A = saddle.solve_suspension(s)
        print(f"{s.name}: {s.n_bead} beads, residual {r:.2e} ({time.time() - t:.1f} s)", flush=True)
        out[f"U_{k}"] = U
        out[f"digest_{k}"] = np.array(digest(s))
    np.savez(os.path.join(HERE, "uneven8_oracle.npz"), picks=np.array(UNEVEN_PICK), **out)


def request():
    """One Brownian solve of a serving request (kT = 1, dt = 1e-3, shear rate 1, splitting
    parameter 25/L) given its real-space and near-field noise (grid noise zero): the
    real-space root by eigendecomposition of the PSE real part, summed to a cutoff of
    6/xi (its functions are below 1e-14 of the self mobility there); the near-field root
    by REQUEST_LANCZOS_STEPS Lanczos steps."""
    s = fsdgen.serving_request(REQUEST_PICK, kT=1.0, shear_rate=1.0)
    xi = 25.0 / s.L
    psi_r, psi_nf = fsdgen.brownian_noise(s.n_bead, REQUEST_NOISE_SEED)
    t = time.time()
    A = saddle.assemble(s.L, s.a, s.eta, s.offsets, s.x_body, s.com, s.quat, s.force, s.grad_u, r_lub=s.r_lub)
    body = rigid.body_index(s.offsets)
    ub = brownian.real_space_slip(A.x, s.L, s.a, s.eta, xi, 6.0 / xi, psi_r, s.kT, s.dt)
    fb = np.zeros((s.n_bead, 6))
    fb[:, :3] = brownian.near_field_force(A.x, body, s.L, s.a, s.eta, s.r_lub, psi_nf, s.kT, s.dt,
                                          lanczos_steps=REQUEST_LANCZOS_STEPS)
    U, F, r, _ = saddle.solve(s.L, s.a, s.eta, s.offsets, s.x_body, s.com, s.quat, s.force, s.grad_u,
                              r_lub=s.r_lub, u_brown=ub, f_brown_nf=fb)
    print(f"{s.name}: {s.n_bead} beads, residual {r:.2e} ({time.time() - t:.1f} s)", flush=True)
    np.savez(os.path.join(HERE, "request27_oracle.npz"), digest=np.array(digest(s)), U=U, residual=r, xi=xi,
             lanczos_steps=REQUEST_LANCZOS_STEPS)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "doublets"
    if which == "doublets":
        run(0, 1, "doublets16_oracle.npz")
    elif which == "clusters":
        run(1, 10, "clusters256x8_oracle.npz")
    elif which == "c3sub":
        c3_sub()
    elif which == "uneven":
        uneven()
    elif which == "request":
        request()
    else:
        raise SystemExit(f"unknown workload {which}")
