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


def test_median_correlation_skips_nodes_whose_qoi_does_not_vary():
    # 6 clamped nodes (Q_H identically 0, rho undefined and returned as 0)
    # and 4 varying nodes with a near-perfect surrogate: over all 10 nodes
    # the median would be 0 and the rule would fall back; over the varying
    # ones it is ~1 and the control variate is used.
    rng = np.random.default_rng(6)
    N, M = 64, 4096
    qH = np.zeros((10, N))
    qH[6:] = 2.0 + rng.standard_normal((4, N))
    qL = qH + 1e-3 * rng.standard_normal((10, N))
    qL[:6] = rng.standard_normal((6, N))            # surrogate noise where Q_H is constant
    sumL = qL.sum(1) * (M / N)
    sumsqL = (qL ** 2).sum(1) * (M / N)
    r = cv.cv_moments(qH, qL, sumL, sumsqL, M)
    assert np.all(r["rho"][:6] == 0.0) and np.all(r["rho"][6:] > 0.99)
    assert not cv.use_control_variate(r["rho"], 0.01)                       # all nodes: median 0
    assert cv.use_control_variate(r["rho"], 0.01, varying=cv.plain_moments(qH)[1] > 0)
    m, v, used = cv.estimate(qH, qL, sumL, sumsqL, M, 0.01)
    assert used
    # at the constant nodes beta = 0, so the estimate is the plain one: 0
    assert np.all(m[:6] == 0.0) and np.all(v[:6] == 0.0)
    # no varying node at all: plain statistics
    m0, v0, used0 = cv.estimate(np.zeros((3, N)), qL[:3], sumL[:3], sumsqL[:3], M, 0.01)
    assert not used0 and np.all(m0 == 0.0) and np.all(v0 == 0.0)
