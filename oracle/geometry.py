"""Geometry update with selective stiffness refresh (Sec. 2.3) -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

The lumen geometry moves with the displacement, and the stiffness is
rebuilt from the moved geometry only every few steps (the displacements stay
small, so the matrix changes little between refreshes).  Per sample s, with
m = every * floor(n / every) the last refresh step,

    K_m = sum_e (E h)_{e,s} P_e^T Khat_e(x + u_m) P_e,
    R_n = R_m + K_m (u_n - u_m),     R_m = R_{m'} + K_{m'} (u_m - u_{m'}),

with Khat_e(.) the element matrix of Sec. 2.2.1 evaluated on the moved node
coordinates, u_0 = 0, R_0 = 0 (the first interval is the linear model).
The internal force is carried incrementally: at a refresh the force is the
same with the old and the new matrix, and the matrix only acts on the
displacement since the last refresh.  (Applying a refreshed matrix to the
total displacement, K_m u_n, makes the force jump at every refresh; in this
oracle that variant grows without bound within 2,000 steps at a refresh
every 10 steps even at 2 % strain.)  Masses, the load and the step stay
those of the reference geometry.

Pins (tests/test_oracle_geometry.py): the matrix of a rigidly rotated
geometry is the rotated matrix, a translated or uniformly scaled geometry
gives the same matrix, the patch test holds on a stretched geometry (strain
energy of a linear field = area x the constitutive form of its strains, on
the stretched area), a flat plate stretched uniformly in k refreshed
increments carries on its edge the sum of the increments' homogeneous
edge tractions, each on the plate as stretched before it (closed form,
which the total-displacement form K_m u_n misses), a run with refreshes
equals plain runs of the stepper chained segment by segment with the force
base and the matrix moved in between, and at a vanishing load the run
tends to the linear one.
"""
from __future__ import annotations

import numpy as np

from . import assembly, element


class IncrementalForce:
    """Internal force carried across stiffness refreshes.

    force(u) = R_m + K_m (u - u_m); refresh(u) first moves the base to the
    force at u, R_m <- R_m + K_m (u - u_m), u_m <- u, and then rebuilds the
    matrix on the moved geometry, K_m <- K_at(u).  Without a refresh it is
    the linear force K u (R_m = 0, u_m = 0 by default)."""

    def __init__(self, K, K_at=None, R_base=None, u_base=None):
        n = K.shape[0]
        self.K = K
        self.K_at = K_at
        self.R_base = np.zeros(n) if R_base is None else np.array(R_base, dtype=np.float64)
        self.u_base = np.zeros(n) if u_base is None else np.array(u_base, dtype=np.float64)

    def force(self, u: np.ndarray) -> np.ndarray:
        return self.R_base + self.K @ (u - self.u_base)

    def refresh(self, u: np.ndarray) -> None:
        self.R_base = self.force(u)
        self.u_base = np.array(u, dtype=np.float64)
        self.K = self.K_at(self.u_base)


def deformed_stiffness(xyz: np.ndarray, tri: np.ndarray, u: np.ndarray, eh_col: np.ndarray, nu: float,
                       shear_k: float):
    """K(x + u) for one sample: u [n_dof] (node-major), eh_col [n_el]."""
    khat, _, _ = element.reference_stiffness(xyz + u.reshape(-1, 3), tri, nu, shear_k)
    return assembly.assemble_stiffness(tri, khat, eh_col, xyz.shape[0])
