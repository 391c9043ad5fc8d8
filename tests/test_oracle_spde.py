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


def test_sampled_fields_have_the_discrete_and_matern_variance():
    """8,192 fields drawn through spde.sample on a flat 12 x 12 square
    (spacing 0.2, kappa = sqrt 2): at the middle node the empirical
    variance lies within 4 standard errors of the discrete variance
    sum_k (K^-1 e_c)_k^2 C~_k, the continuous Matern variance
    1 / (4 pi kappa^2) within the discretisation error (3.9 % at this
    spacing) plus 4 standard errors, and the empirical correlation with the
    node at distance rho within 4 standard errors of kappa rho K_1(kappa rho)
    (white-noise scaling C~^(1/2): C~_k = 0.04 inside, so a missing or
    squared root moves the variance by a factor 25)."""
    kappa = math.sqrt(2.0)
    n, side = 61, 12.0
    xyz, tri = _square(n, side)
    c = (n // 2) * n + n // 2
    rho = math.sqrt(8.0) / kappa
    j = c + int(round(rho / (side / (n - 1))))
    rng = np.random.default_rng(21)
    N, chunk = 8192, 1024
    xc, xj = [], []
    for _ in range(N // chunk):
        x = spde.sample(xyz, tri, rng.standard_normal((n * n, chunk)), kappa)
        xc.append(x[c])
        xj.append(x[j])
    xc, xj = np.concatenate(xc), np.concatenate(xj)
    K, C = spde.operator(xyz, tri, kappa)
    w = spla.splu(K.tocsc()).solve(np.eye(1, n * n, c).ravel())
    var_discrete = float(np.sum(w * w * C))
    se = var_discrete * math.sqrt(2.0 / (N - 1))
    var_emp = float(np.mean(xc * xc))
    assert abs(np.mean(xc)) < 4.0 * math.sqrt(var_discrete / N)
    assert abs(var_emp - var_discrete) < 4.0 * se
    var_matern = spde.marginal_variance(kappa)
    assert abs(var_emp - var_matern) < 0.039 * var_matern + 4.0 * se
    d = np.linalg.norm(xyz[j] - xyz[c])
    r_expect = kappa * d * special.k1(kappa * d)
    r_emp = float(np.mean(xc * xj) / math.sqrt(np.mean(xc * xc) * np.mean(xj * xj)))
    assert abs(r_emp - r_expect) < 4.0 * (1.0 - r_expect ** 2) / math.sqrt(N) + 0.01
