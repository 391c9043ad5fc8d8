"""Pins for the control-variate estimator and its fallback."""
import numpy as np

from oracle import control_variate as cv


def test_gaussian_toy_unbiased_and_variance_formula():
    rng = np.random.default_rng(3)
    mu, N, M, sig_n, trials = 1.7, 64, 4096, 0.5, 3000
    est = np.empty(trials)
    plain = np.empty(trials)
    for t in range(trials):
        X = mu + rng.standard_normal((1, N))
        L = X + sig_n * rng.standard_normal((1, N))
        Lp = mu + rng.standard_normal(M) + sig_n * rng.standard_normal(M)
        r = cv.cv_moments(X, L, np.array([Lp.sum()]), np.array([(Lp ** 2).sum()]), M)
        est[t] = r["mean"][0]
        plain[t] = X.mean()
    rho = 1.0 / np.sqrt(1.0 + sig_n ** 2)
    se = est.std() / np.sqrt(trials)
    assert abs(est.mean() - mu) < 3.5 * se
    predicted = (1.0 / N) * cv.predicted_variance_ratio(rho, N, M)
    # finite-N estimate of beta inflates the variance by ~1/(N-3); allow 15 %
    assert abs(est.var() / predicted - 1.0) < 0.15
    assert est.var() < 0.35 * plain.var()


def test_perfect_surrogate_exact_moments():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((5, 32)) * 2 + 3
    # exact low-fidelity moments of a large independent sample set equal to
    # the true mean 3 and second moment 4 + 9
    M = 10 ** 6
    r = cv.cv_moments(X, X.copy(), np.full(5, 3.0 * M), np.full(5, 13.0 * M), M)
    assert np.allclose(r["mean"], 3.0, atol=1e-12)
    assert np.allclose(r["var"], 4.0, atol=1e-10)
    assert np.allclose(r["rho"], 1.0) and np.allclose(r["beta"], 1.0)


def test_fallback_returns_plain_statistics():
    rng = np.random.default_rng(5)
    qH = rng.standard_normal((7, 40))
    junk = rng.standard_normal((7, 40))          # uncorrelated "surrogate"
    m, v, used = cv.estimate(qH, junk, junk.sum(1) * 10, (junk ** 2).sum(1) * 10, 400, 0.5)
    assert not used
    pm, pv = cv.plain_moments(qH)
    assert np.array_equal(m, pm) and np.array_equal(v, pv)
    m2, v2, used2 = cv.estimate(qH, qH + 1e-3 * junk, qH.sum(1) * 10, (qH ** 2).sum(1) * 10, 400, 0.01)
    assert used2
