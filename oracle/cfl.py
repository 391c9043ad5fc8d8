"""Stable explicit time step from the element eigenvalue bound -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Central differences are stable for omega_max dt < 2 (undamped; mass
proportional damping treated by eq. dynamicsCD leaves the limit unchanged).
The paper sets the step from a CFL wave-speed argument (Sec. 1) scaled by
0.9.  Here omega_max^2 of the assembled pencil (K_s, M_s) is bounded by the
largest element eigenvalue (Irons-Treharne): with the element's share of the
lumped mass rho h_{e,s} A_e / 3 on each of its nodes,

    lambda(K_{e,s}, M_{e,s}) = 3 E_{e,s} lambda_max(Khat_e) / (rho A_e),

and dt = safety * 2 / sqrt(max_{e,s} of that), one step for the whole
ensemble.

Pins (tests/test_oracle_cfl.py): the global generalized eigenvalue never
exceeds the bound; the undamped scheme stays bounded at 0.99 * 2/omega_glob
and diverges at 1.05 * 2/omega_glob.
"""
from __future__ import annotations

import numpy as np


def element_lambda_max(khat: np.ndarray) -> np.ndarray:
    """Largest eigenvalue of each symmetric 9x9 Khat_e."""
    return np.linalg.eigvalsh(khat)[:, -1]


def omega2_bound(khat: np.ndarray, area: np.ndarray, eh: np.ndarray, h: np.ndarray, rho: float) -> float:
    lam = element_lambda_max(khat)
    E = eh / h
    return float(np.max(3.0 * E * (lam / (rho * area))[:, None]))


def stable_dt(khat, area, eh, h, rho, safety: float = 0.9) -> float:
    return safety * 2.0 / np.sqrt(omega2_bound(khat, area, eh, h, rho))
