"""CPU oracle for the rigid-aggregate saddle-point solve.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's CPU
baseline leg may import this package.  The product path never calls it and
shares no code with it.

Everything here is plain, dense and FP64:

* rpy      -- free-space force-torque RPY blocks (closed forms) and the periodic
              mobility assembled densely by a Beenakker-split Ewald sum
              (real-space images + a direct wave-vector sum, no grid).
* lub      -- the stated near-field lubrication model, assembled densely.
* rigid    -- the geometric constraint matrix Sigma, bead positions from
              quaternions, the right-hand side of the aggregate saddle system.
* saddle   -- direct solves of the saddle system (Schur + Cholesky, full LU),
              the dense block-triangular preconditioner and a textbook GMRES.
* pse      -- the positively split Ewald decomposition evaluated by quadrature
              and a direct k-sum, for checking the two halves separately.
* integrate -- explicit Euler update of centroids and quaternions.
* brownian -- the Brownian right-hand-side terms with exact (eigendecomposition)
              square roots of the real-space mobility and the lubrication matrix.
* stress   -- the constraint stresslet of each aggregate from the solved bead forces.

Paper sections cited are those of "Fast Stokesian Dynamics for Rigid
Aggregates" (Mangal et al.).
"""
from . import rpy, lub, rigid, saddle, integrate, pse, brownian, forces, drift, stress  # noqa: F401
