"""Matern covariance and dense-Cholesky Gaussian fields -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Matern covariance (Sec. 2.1):
    r(d) = sigma^2 / (2^(nu-1) Gamma(nu)) (kappa d)^nu K_nu(kappa d),
    correlation length rho = sqrt(8 nu) / kappa,
with K_nu the modified Bessel function of the second kind and d the
Euclidean distance in R^3.

Fields for tiny meshes: the covariance of the element centroids,
Sigma = L L^T by a dense Cholesky, and independent standard-normal draws z_E,
z_h (the paper writes "the same z" for both fields; independent draws are
used so E and h are not perfectly correlated):
    log E = log E_mean + L z_E,   log h = log h_mean + L z_h,
(E h)_{e,s} = E_{e,s} h_{e,s}.  The paper uses Gaussian marginals; the
workloads here use lognormal ones (Gaussian log-fields).

Pins (tests/test_oracle_matern.py): r(0) = sigma^2; the textbook closed
forms for nu = 1/2 (sigma^2 e^{-kappa d}) and nu = 3/2
(sigma^2 (1 + kappa d) e^{-kappa d}); Sigma positive definite with
diag = sigma^2; the empirical covariance of many samples within sampling
error of Sigma.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def covariance(d: np.ndarray, sigma: float, nu: float, rho: float) -> np.ndarray:
    kappa = math.sqrt(8.0 * nu) / rho
    x = kappa * np.asarray(d, dtype=np.float64)
    r = np.empty_like(x)
    zero = x == 0.0
    r[zero] = sigma * sigma
    xp = x[~zero]
    r[~zero] = sigma * sigma / (2.0 ** (nu - 1.0) * special.gamma(nu)) * xp ** nu * special.kv(nu, xp)
    return r


def centroid_covariance(xyz: np.ndarray, tri: np.ndarray, sigma: float, nu: float, rho: float) -> np.ndarray:
    c = (xyz[tri[:, 0]] + xyz[tri[:, 1]] + xyz[tri[:, 2]]) / 3.0
    d = np.sqrt(np.sum((c[:, None, :] - c[None, :, :]) ** 2, axis=-1))
    return covariance(d, sigma, nu, rho)


def cholesky_factor(Sigma: np.ndarray) -> np.ndarray:
    try:
        return np.linalg.cholesky(Sigma)
    except np.linalg.LinAlgError:
        jitter = 1e-12 * float(np.max(np.diag(Sigma)))
        return np.linalg.cholesky(Sigma + jitter * np.eye(Sigma.shape[0]))


def lognormal_fields(xyz: np.ndarray, tri: np.ndarray, S: int, seed: int, E_mean: float = 7.0e6,
                     h_mean: float = 0.1, sigma_log: float = 0.2, rho: float = 2.0, nu: float = 1.0):
    """(E h) [n_el, S] and h [n_el, S] on element centroids."""
    L = cholesky_factor(centroid_covariance(xyz, tri, sigma_log, nu, rho))
    rng = np.random.default_rng(seed)
    zE = rng.standard_normal((tri.shape[0], S))
    zh = rng.standard_normal((tri.shape[0], S))
    E = np.exp(math.log(E_mean) + L @ zE)
    h = np.exp(math.log(h_mean) + L @ zh)
    return E * h, h
