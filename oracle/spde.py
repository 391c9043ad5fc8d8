"""Gaussian Markov random field samples from the SPDE formulation of the
Matern field (Sec. 2.1) -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

With piecewise linear basis functions on the surface triangles, C_ij =
<psi_i, psi_j> lumped to the diagonal C~_ii = sum_{e containing i} A_e / 3,
and G_ij = <grad psi_i, grad psi_j> (per element A_e grad psi_a . grad psi_b
with the in-plane gradients of the linear triangle).  For alpha = 2 (Matern
nu = 1 on a surface, d = 2) the precision is Q = K C~^-1 K with
K = kappa^2 C~ + G, so x = K^-1 C~^(1/2) z with z standard normal has
covariance Q^-1.  The continuous field's marginal variance is
Gamma(nu) / (Gamma(nu + d/2) (4 pi)^(d/2) kappa^(2 nu)) = 1 / (4 pi kappa^2).

Pins (tests/test_oracle_spde.py): G annihilates constants, is symmetric and
positive semi-definite; the lumped masses add up to the surface area; the
Dirichlet energy of a linear function on a flat patch is |a|^2 times the
area; at the middle of a large flat square the discrete field's variance
and its correlation at the correlation length rho = sqrt(8) / kappa match
the Matern values 1 / (4 pi kappa^2) and kappa rho K_1(kappa rho).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import element


def laplace_matrices(xyz: np.ndarray, tri: np.ndarray):
    """Lumped mass diagonal C~ [n_nodes] and stiffness G (CSR) of the
    surface Laplacian with piecewise linear elements."""
    n = xyz.shape[0]
    p1, p2, p3 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    _, x, y = element.local_frames(p1, p2, p3)
    A = element.areas(x, y)
    B = element.strain_matrix(x, y, A)
    gx = B[:, 0, 0::3]                     # d psi_j / dx, j = 1..3
    gy = B[:, 1, 1::3]                     # d psi_j / dy
    Ge = A[:, None, None] * (gx[:, :, None] * gx[:, None, :] + gy[:, :, None] * gy[:, None, :])
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    G = sp.coo_matrix((Ge.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    C = np.zeros(n)
    for a in range(3):
        np.add.at(C, tri[:, a], A / 3.0)
    return C, G


def operator(xyz: np.ndarray, tri: np.ndarray, kappa: float):
    """K = kappa^2 C~ + G (CSR) and C~."""
    C, G = laplace_matrices(xyz, tri)
    return (sp.diags(kappa * kappa * C) + G).tocsr(), C


def sample(xyz: np.ndarray, tri: np.ndarray, z: np.ndarray, kappa: float) -> np.ndarray:
    """x = K^-1 C~^(1/2) z for white noise z [n_nodes, S] (direct solve)."""
    K, C = operator(xyz, tri, kappa)
    rhs = np.sqrt(C)[:, None] * z
    return spla.splu(K.tocsc()).solve(rhs)


def marginal_variance(kappa: float) -> float:
    """1 / (4 pi kappa^2): nu = 1, d = 2."""
    return 1.0 / (4.0 * math.pi * kappa * kappa)
