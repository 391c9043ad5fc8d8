"""The learned form's host-side fallback rule (no GPU): the per-node
control-variate kernel is replaced by the oracle's, so only the rule that
picks the control variate or the plain statistics is under test."""
import numpy as np
import pytest

from oracle import control_variate as cv
from paper_2101_09059_amd import learned


@pytest.fixture
def oracle_kernel(monkeypatch):
    def cv_moments(qH, qL, sumL, sumsqL, M, device=0):
        r = cv.cv_moments(qH, qL, sumL, sumsqL, M)
        return r["mean"], r["var"], r["rho"]
    monkeypatch.setattr(learned.ensfem, "cv_moments", cv_moments)


def _case(seed, noise, n_const=6, n_var=5, N=64, M=4096):
    rng = np.random.default_rng(seed)
    qH = np.zeros((n_const + n_var, N))
    qH[n_const:] = 1.0 + rng.standard_normal((n_var, N))
    qL = qH + noise * rng.standard_normal(qH.shape)
    return qH, qL, qL.sum(1) * (M / N), (qL ** 2).sum(1) * (M / N), M


@pytest.mark.parametrize("noise,rmse", [(1e-3, 0.01), (1e-3, 0.2), (3.0, 0.01)])
def test_fallback_rule_matches_the_oracle(oracle_kernel, noise, rmse):
    qH, qL, s1, s2, M = _case(11, noise)
    pm, pv = cv.plain_moments(qH)
    got = learned.estimate(qH, pm, pv, qL, s1, s2, M, rmse)
    m, v, used = cv.estimate(qH, qL, s1, s2, M, rmse)
    assert got["used_cv"] == used
    assert np.array_equal(got["mean"], m) and np.array_equal(got["var"], v)


def test_constant_nodes_do_not_pull_the_median_down(oracle_kernel):
    # more clamped nodes than varying ones, good surrogate: still used
    qH, qL, s1, s2, M = _case(12, 1e-3, n_const=9, n_var=3)
    pm, pv = cv.plain_moments(qH)
    got = learned.estimate(qH, pm, pv, qL, s1, s2, M, 0.01)
    assert got["used_cv"] and got["rho_median"] > 0.99
