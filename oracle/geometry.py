"""Geometry update with selective stiffness refresh (Sec. 2.3) -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

The lumen geometry moves with the displacement, and the stiffness is
rebuilt from the moved geometry only every few steps (the displacements stay
small, so the matrix changes little between refreshes).  Per sample s the
matrix used at step n is

    K_s(x + u_{s,m}) = sum_e (E h)_{e,s} P_e^T Khat_e(x + u_{s,m}) P_e,
    m = every * floor(n / every),

with Khat_e(.) the element matrix of Sec. 2.2.1 evaluated on the moved
node coordinates and u_{s,0} = 0 (the first interval runs on the reference
geometry).  Masses, the load and the step stay those of the reference
geometry; the force is K(x + u_m) u_n with the total displacement u_n.

Pins (tests/test_oracle_geometry.py): the matrix of a rigidly rotated
geometry is the rotated matrix, a translated or uniformly scaled geometry
gives the same matrix, the patch test holds on a stretched geometry (strain
energy of a linear field = area x the constitutive form of its strains, on
the stretched area), and a run with refreshes equals plain runs of the
stepper chained segment by segment with the matrix rebuilt in between.
"""
from __future__ import annotations

import numpy as np

from . import assembly, element


def deformed_stiffness(xyz: np.ndarray, tri: np.ndarray, u: np.ndarray, eh_col: np.ndarray, nu: float,
                       shear_k: float):
    """K(x + u) for one sample: u [n_dof] (node-major), eh_col [n_el]."""
    khat, _, _ = element.reference_stiffness(xyz + u.reshape(-1, 3), tri, nu, shear_k)
    return assembly.assemble_stiffness(tri, khat, eh_col, xyz.shape[0])
