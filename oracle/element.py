"""Three-dof shell element of the wall model (Sec. 2.2.1) -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Per triangle (p1, p2, p3):
  * local frame: e_x along p2 - p1, e_z the unit normal of (p2-p1)x(p3-p1),
    e_y = e_z x e_x (the paper states quantities in a local shell frame but
    does not write the rotation; the in-plane axis choice is immaterial for
    an isotropic material);
  * local coordinates (x_j, y_j) of the nodes relative to p1, area A_e;
  * B, the 5x9 strain-displacement matrix of the linear triangle with rows
    du_x/dx, du_y/dy, gamma_xy, du_z/dx, du_z/dy (Sec. 2.2.1, B equation);
  * C = E/(1-nu^2) * [[1,nu],[nu,1]] (+) (1-nu)/2 (+) k(1-nu)/2 (+) k(1-nu)/2,
    eps_zz = 0 (Sec. 2.2.1, constitutive equation);
  * element stiffness k_e = B^T C B A_e * sum_g w_g zeta_g (E_g): with B
    constant, E and thickness entering only as the scalar (E h)_e, so
    k_e = (E h)_e * Khat_e with Khat_e = A_e * B^T (C/E) B (Sec. 2.2.1,
    stiffness equation);
  * rotated to the global frame: Khat^g = T^T Khat^l T, T = diag(R, R, R)
    with R's rows e_x, e_y, e_z.

Pins (tests/test_oracle_element.py): symmetry, positive semi-definiteness,
rank 5 for k > 0 and 3 for k = 0, zero force under rigid translations (any
k) and infinitesimal rotations (k = 0), invariance under cyclic node
relabelling and rigid rotation of the triangle, and the constant-strain
patch test 1/2 u^T Khat u = 1/2 A eps^T Chat eps for linear displacement
fields with analytically known strains.
"""
from __future__ import annotations

import numpy as np


def local_frames(p1: np.ndarray, p2: np.ndarray, p3: np.ndarray):
    """Rotation rows [m, 3, 3] (e_x, e_y, e_z) and local node coordinates
    x, y [m, 3] (node 1 at the origin)."""
    a = p2 - p1
    b = p3 - p1
    ex = a / np.linalg.norm(a, axis=-1, keepdims=True)
    n = np.cross(a, b)
    ez = n / np.linalg.norm(n, axis=-1, keepdims=True)
    ey = np.cross(ez, ex)
    Rm = np.stack([ex, ey, ez], axis=-2)
    d = np.stack([np.zeros_like(a), a, b], axis=-2)            # [m, 3 nodes, 3]
    x = np.einsum("mjk,mk->mj", d, ex)
    y = np.einsum("mjk,mk->mj", d, ey)
    return Rm, x, y


def areas(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """A_e = 1/2 (x2 y3 - x3 y2) with node 1 at the local origin."""
    return 0.5 * (x[:, 1] * y[:, 2] - x[:, 2] * y[:, 1])


def strain_matrix(x: np.ndarray, y: np.ndarray, A: np.ndarray) -> np.ndarray:
    """B [m, 5, 9] as printed in Sec. 2.2.1, x_ij = x_i - x_j."""
    m = x.shape[0]
    y23 = y[:, 1] - y[:, 2]
    y31 = y[:, 2] - y[:, 0]
    y12 = y[:, 0] - y[:, 1]
    x32 = x[:, 2] - x[:, 1]
    x13 = x[:, 0] - x[:, 2]
    x21 = x[:, 1] - x[:, 0]
    B = np.zeros((m, 5, 9))
    dx = (y23, y31, y12)     # d N_j / dx times 2A
    dy = (x32, x13, x21)     # d N_j / dy times 2A
    for j in range(3):
        B[:, 0, 3 * j + 0] = dx[j]
        B[:, 1, 3 * j + 1] = dy[j]
        B[:, 2, 3 * j + 0] = dy[j]
        B[:, 2, 3 * j + 1] = dx[j]
        B[:, 3, 3 * j + 2] = dx[j]
        B[:, 4, 3 * j + 2] = dy[j]
    return B / (2.0 * A)[:, None, None]


def constitutive_unit(nu: float, shear_k: float) -> np.ndarray:
    """C / E (5x5), Sec. 2.2.1."""
    c = np.zeros((5, 5))
    c[0, 0] = c[1, 1] = 1.0
    c[0, 1] = c[1, 0] = nu
    c[2, 2] = 0.5 * (1.0 - nu)
    c[3, 3] = c[4, 4] = 0.5 * shear_k * (1.0 - nu)
    return c / (1.0 - nu * nu)


def reference_stiffness(xyz: np.ndarray, tri: np.ndarray, nu: float, shear_k: float):
    """Khat_e in the global frame [m, 9, 9] (dof order u_x1,u_y1,u_z1,u_x2,...),
    areas A_e [m] and unit normals [m, 3]."""
    p1, p2, p3 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    Rm, x, y = local_frames(p1, p2, p3)
    A = areas(x, y)
    if np.any(~(A > 0.0)):
        raise ValueError("degenerate or inverted triangle")
    B = strain_matrix(x, y, A)
    C = constitutive_unit(nu, shear_k)
    k_loc = A[:, None, None] * np.einsum("mai,ab,mbj->mij", B, C, B)
    T = np.zeros((tri.shape[0], 9, 9))
    for j in range(3):
        T[:, 3 * j:3 * j + 3, 3 * j:3 * j + 3] = Rm
    k_glob = np.einsum("mai,mab,mbj->mij", T, k_loc, T)
    return k_glob, A, Rm[:, 2, :]
