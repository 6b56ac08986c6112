"""Write oracle reference values for the full-size parity workloads.

Calls only the CPU oracle and the seeded generator.  Each output stores a
digest of the generated inputs so a test can confirm it regenerates the same
system before comparing.

    python tests/golden/make_golden.py doublets      # 16 doublets, one solve
    python tests/golden/make_golden.py clusters      # 256 x 8 clusters, 10 steps
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
from oracle import integrate, saddle  # noqa: E402


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


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "doublets"
    if which == "doublets":
        run(0, 1, "doublets16_oracle.npz")
    elif which == "clusters":
        run(1, 10, "clusters256x8_oracle.npz")
    else:
        raise SystemExit(f"unknown workload {which}")
