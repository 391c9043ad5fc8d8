"""Per-sample global stiffness and lumped mass -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

K_s = sum_e (E h)_{e,s} P_e^T Khat_e P_e, assembled for ONE sample at a time
as a scipy CSR matrix (the plain definition: no ensemble batching, no
element-by-element product).  dof numbering: 3*node + component.

Lumped mass (Sec. 2.3, lumped M pre-assembled before the time loop): the
shell mass rho h_{e,s} A_e is split equally over the three element nodes,
m_{i,s} = sum_{e ni i} rho h_{e,s} A_e / 3, the same on the node's three dofs.

Pins: symmetry and u^T(Kv) = v^T(Ku) on random vectors, translation
null-space of the unclamped matrix, and the clamped-cylinder Laplace law
(tests/test_oracle_assembly.py, tests/test_oracle_static.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def element_dofs(tri: np.ndarray) -> np.ndarray:
    """[m, 9] global dof indices of each element's nine dofs."""
    return (3 * tri[:, :, None] + np.arange(3)[None, None, :]).reshape(tri.shape[0], 9)


def assemble_stiffness(tri: np.ndarray, khat: np.ndarray, eh_col: np.ndarray, n_nodes: int) -> sp.csr_matrix:
    """K for one sample: eh_col [m] scales each element's Khat."""
    dofs = element_dofs(tri)
    rows = np.repeat(dofs, 9, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 9)).reshape(-1)
    vals = (eh_col[:, None, None] * khat).reshape(-1)
    n = 3 * n_nodes
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K


def lumped_mass(tri: np.ndarray, area: np.ndarray, h_col: np.ndarray, rho: float, n_nodes: int,
                scale_col: np.ndarray = None) -> np.ndarray:
    """Nodal lumped mass [n_nodes] for one sample; scale_col [n_el]: optional
    per-element density factors (mass scaling)."""
    me = rho * h_col * area / 3.0
    if scale_col is not None:
        me = rho * scale_col * h_col * area / 3.0
    m = np.zeros(n_nodes)
    for a in range(3):
        np.add.at(m, tri[:, a], me)
    return m
