"""Multifidelity control-variate estimator -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

High fidelity Q_H (the plain solver) and low fidelity Q_L (the surrogate)
on the same N inputs, plus M further low-fidelity draws Q_L' on fresh
inputs.  Per node:
    beta = Cov_N(Q_H, Q_L) / Var_N(Q_L)
    mu   = mean_N(Q_H) - beta (mean_N(Q_L) - mean_M(Q_L'))
and the same estimator on the squares gives the second moment m2, from
which var = m2 - mu^2.  With correlation rho between the fidelities the
estimator's variance is (sigma_H^2 / N) (1 - rho^2 M / (M + N)).

The estimator is used only when the surrogate earns it: median per-node
correlation >= 0.9 and held-out relative RMSE <= 5 %; otherwise the plain
N-sample statistics are returned unchanged.  The correlation is undefined
at nodes whose high-fidelity QoI does not vary (the clamped rings), so the
median runs over the varying nodes only.

Pins (tests/test_oracle_control_variate.py): a Gaussian toy (H = X,
L = X + sigma Z) where repeated trials show the estimator unbiased and its
variance equal to the formula above; a perfect surrogate with exact
low-fidelity moments recovers the exact mean; the fallback returns the
plain statistics bit for bit; constant nodes do not enter the median.
"""
from __future__ import annotations

import numpy as np


def plain_moments(qH: np.ndarray):
    """Per-row mean and unbiased variance of [n, N] samples."""
    N = qH.shape[1]
    mean = qH.sum(axis=1) / N
    d = qH - mean[:, None]
    return mean, (d * d).sum(axis=1) / (N - 1)


def _cv(h, l, l_mean_M):
    N = h.shape[1]
    hm = h.sum(axis=1) / N
    lm = l.sum(axis=1) / N
    dh = h - hm[:, None]
    dl = l - lm[:, None]
    cov = (dh * dl).sum(axis=1) / (N - 1)
    var_l = (dl * dl).sum(axis=1) / (N - 1)
    var_h = (dh * dh).sum(axis=1) / (N - 1)
    beta = np.where(var_l > 0, cov / np.where(var_l > 0, var_l, 1.0), 0.0)
    rho = np.where((var_l > 0) & (var_h > 0), cov / np.sqrt(np.where(var_l > 0, var_l, 1.0) *
                                                              np.where(var_h > 0, var_h, 1.0)), 0.0)
    return hm - beta * (lm - l_mean_M), beta, rho


def cv_moments(qH: np.ndarray, qL: np.ndarray, sumL_M: np.ndarray, sumsqL_M: np.ndarray, M: int):
    """Control-variate mean and variance per node.  qH, qL [n, N] paired;
    sumL_M, sumsqL_M [n]: sums of Q_L' and Q_L'^2 over the M fresh draws."""
    mu, beta, rho = _cv(qH, qL, sumL_M / M)
    m2, _, _ = _cv(qH * qH, qL * qL, sumsqL_M / M)
    return dict(mean=mu, var=m2 - mu * mu, beta=beta, rho=rho)


def predicted_variance_ratio(rho, N: int, M: int):
    return 1.0 - rho * rho * M / (M + N)


def use_control_variate(rho: np.ndarray, heldout_rel_rmse: float, rho_min: float = 0.9,
                        rmse_max: float = 0.05, varying=None) -> bool:
    """The fallback rule; varying (bool per node) marks the nodes whose
    high-fidelity QoI varies, the only ones where rho is defined (all nodes
    when None).  No varying node: plain statistics."""
    r = rho if varying is None else rho[varying]
    if r.size == 0:
        return False
    return bool(np.median(r) >= rho_min and heldout_rel_rmse <= rmse_max)


def estimate(qH, qL, sumL_M, sumsqL_M, M, heldout_rel_rmse):
    """The estimator with its fallback: returns (mean, var, used_cv)."""
    cv = cv_moments(qH, qL, sumL_M, sumsqL_M, M)
    mean, var = plain_moments(qH)
    if use_control_variate(cv["rho"], heldout_rel_rmse, varying=var > 0):
        return cv["mean"], cv["var"], True
    return mean, var, False
