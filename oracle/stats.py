"""Per-node ensemble statistics -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

mean_i = (1/S) sum_s q_{i,s};  var_i = 1/(S-1) sum_s (q_{i,s} - mean_i)^2
(unbiased), two-pass.  Pinned against hand-computed values on a small
array (tests/test_oracle_stats.py).
"""
from __future__ import annotations

import numpy as np


def moments(q: np.ndarray):
    S = q.shape[1]
    mean = np.sum(q, axis=1) / S
    d = q - mean[:, None]
    var = np.sum(d * d, axis=1) / (S - 1)
    return mean, var
