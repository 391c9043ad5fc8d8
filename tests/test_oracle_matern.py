"""Pins for the Matern covariance and the dense-Cholesky field sampler (Sec. 2.1)."""
import math

import numpy as np

from oracle import matern
from paper_2101_09059_amd import inputs


def test_closed_forms():
    d = np.linspace(0.0, 5.0, 41)
    s, rho = 0.7, 1.3
    # nu = 1/2: exponential covariance; nu = 3/2: (1 + x) e^{-x}
    k = math.sqrt(8 * 0.5) / rho
    assert np.allclose(matern.covariance(d, s, 0.5, rho), s * s * np.exp(-k * d), rtol=1e-13, atol=0)
    k = math.sqrt(8 * 1.5) / rho
    assert np.allclose(matern.covariance(d, s, 1.5, rho), s * s * (1 + k * d) * np.exp(-k * d),
                       rtol=1e-13, atol=0)
    # nu = 1: continuous at 0 with value sigma^2, about 0.1-0.15 correlation at d = rho
    r = matern.covariance(np.array([0.0, 1e-8, 2.0]), 1.0, 1.0, 2.0)
    assert r[0] == 1.0 and abs(r[1] - 1.0) < 1e-12 and 0.1 < r[2] < 0.16


def test_centroid_covariance_pd_and_sampling():
    m = inputs.cylinder(1.0, 10.0, 12, 6)
    Sig = matern.centroid_covariance(m.xyz, m.tri, 0.2, 1.0, 2.0)
    assert np.allclose(np.diag(Sig), 0.04)
    L = matern.cholesky_factor(Sig)
    assert np.max(np.abs(L @ L.T - Sig)) < 1e-14
    N = 20000
    rng = np.random.default_rng(11)
    X = L @ rng.standard_normal((Sig.shape[0], N))
    C = X @ X.T / N
    se = np.sqrt((Sig ** 2 + np.outer(np.diag(Sig), np.diag(Sig))) / N)
    assert np.mean(np.abs(C - Sig) / se) < 1.2
    assert np.max(np.abs(C - Sig) / se) < 5.5


def test_lognormal_fields_reproducible_and_scaled():
    m = inputs.cylinder(1.0, 10.0, 40, 20)
    eh, h = matern.lognormal_fields(m.xyz, m.tri, 8, seed=1)
    eh2, h2 = matern.lognormal_fields(m.xyz, m.tri, 8, seed=1)
    assert np.array_equal(eh, eh2) and np.array_equal(h, h2)
    lh = np.log(h)
    assert abs(np.median(lh) - math.log(0.1)) < 0.2
    assert 0.05 < np.std(lh - lh.mean(axis=0)) < 0.3


def test_circulant_lattice_sampler_matches_matern():
    # the input generator's nodal lattice sampler reproduces the oracle's
    # Matern covariance of the chord distance between nodes
    m = inputs.cylinder(1.0, 10.0, 24, 14)
    rng = np.random.default_rng(12)
    N = 6000
    X = inputs.matern_nodal_lattice(m, N, rng, 0.2, 2.0, 1.0)
    C = X @ X.T / N
    d = np.linalg.norm(m.xyz[:, None, :] - m.xyz[None, :, :], axis=-1)
    Sig = matern.covariance(d, 0.2, 1.0, 2.0)
    se = np.sqrt((Sig ** 2 + np.outer(np.diag(Sig), np.diag(Sig))) / N)
    assert np.mean(np.abs(C - Sig) / se) < 1.2


def test_lognormal_fields_log_means_and_spread():
    """4,096 draws on a 12 x 6 cylinder: per element, the sample means of
    log E = log((E h) / h) and of log h lie within 5 standard errors
    (0.2 / sqrt(S)) of log 7e6 and log 0.1, their variances within 5
    standard errors of 0.2^2, and log E and log h are uncorrelated
    (independent draws)."""
    m = inputs.cylinder(1.0, 10.0, 12, 6)
    S = 4096
    eh, h = matern.lognormal_fields(m.xyz, m.tri, S, seed=31)
    lE, lh = np.log(eh / h), np.log(h)
    se_mean = 0.2 / math.sqrt(S)
    se_var = 0.04 * math.sqrt(2.0 / (S - 1))
    for lf, mu in ((lE, math.log(7.0e6)), (lh, math.log(0.1))):
        assert np.max(np.abs(lf.mean(axis=1) - mu)) < 5.0 * se_mean
        assert abs(lf.mean() - mu) < 5.0 * se_mean
        assert np.max(np.abs(lf.var(axis=1, ddof=1) - 0.04)) < 5.0 * se_var
    cE, ch = lE - lE.mean(axis=1, keepdims=True), lh - lh.mean(axis=1, keepdims=True)
    corr = np.sum(cE * ch, axis=1) / np.sqrt(np.sum(cE * cE, axis=1) * np.sum(ch * ch, axis=1))
    assert np.max(np.abs(corr)) < 5.0 / math.sqrt(S)
