"""Pins of the oracle's SPDE (GMRF) Matern sampler."""
import math

import numpy as np
import scipy.sparse.linalg as spla
from scipy import special

from oracle import spde
from paper_2101_09059_amd import inputs


def _square(n, side):
    """Flat square [0, side]^2 in the xy-plane, n x n nodes, both diagonals
    alternating (no preferred direction)."""
    xs, ys = np.meshgrid(np.linspace(0, side, n), np.linspace(0, side, n))
    xyz = np.stack([xs.ravel(), ys.ravel(), np.zeros(n * n)], 1)
    tri = []
    for j in range(n - 1):
        for i in range(n - 1):
            a = j * n + i
            if (i + j) % 2:
                tri += [(a, a + 1, a + n + 1), (a, a + n + 1, a + n)]
            else:
                tri += [(a, a + 1, a + n), (a + 1, a + n + 1, a + n)]
    return xyz, np.array(tri, dtype=np.int32)


def test_laplacian_structure():
    m = inputs.cylinder(1.0, 3.0, 14, 8)
    C, G = spde.laplace_matrices(m.xyz, m.tri)
    assert np.max(np.abs(G @ np.ones(m.n_nodes))) < 1e-12 * abs(G).max()
    assert abs(G - G.T).max() < 1e-14 * abs(G).max()
    assert np.linalg.eigvalsh(G.toarray())[0] > -1e-12 * abs(G).max()
    p = m.xyz[m.tri]
    area = 0.5 * np.linalg.norm(np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), axis=1).sum()
    assert abs(C.sum() / area - 1.0) < 1e-13


def test_dirichlet_energy_of_a_linear_function():
    xyz, tri = _square(7, 2.0)
    _, G = spde.laplace_matrices(xyz, tri)
    a = np.array([0.7, -1.3])
    f = xyz[:, :2] @ a
    assert abs(f @ (G @ f) / (a @ a * 4.0) - 1.0) < 1e-12


def test_variance_and_correlation_match_matern():
    """Middle of a 24 x 24 square with rho = 2 (kappa = sqrt 2), spacing
    0.08: var(x_c) = sum_k (K^-1 e_c)_k^2 C~_k against 1 / (4 pi kappa^2),
    and the correlation at distance rho against kappa rho K_1(kappa rho)."""
    kappa = math.sqrt(2.0)
    n, side = 301, 24.0
    xyz, tri = _square(n, side)
    K, C = spde.operator(xyz, tri, kappa)
    c = (n // 2) * n + n // 2
    e = np.zeros(n * n)
    e[c] = 1.0
    w = spla.splu(K.tocsc()).solve(e)
    var = float(np.sum(w * w * C))
    assert abs(var / spde.marginal_variance(kappa) - 1.0) < 0.01
    rho = math.sqrt(8.0) / kappa
    j = c + int(round(rho / (side / (n - 1))))            # same row, distance rho
    d = np.linalg.norm(xyz[j] - xyz[c])
    cov = float(np.sum(w * C * spla.splu(K.tocsc()).solve(np.eye(1, n * n, j).ravel())))
    corr = cov / var
    expect = kappa * d * special.k1(kappa * d)
    assert abs(corr - expect) < 0.005
