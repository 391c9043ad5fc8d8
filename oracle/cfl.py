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

Mass scaling (Sec. 1 names it as a way to raise the critical step): for a
target step dt_t, every element and sample whose bound exceeds (2/dt_t)^2
gets its density multiplied by f = lambda dt_t^2 / 4 (f = 1 otherwise), so
its bound lambda / f is at most (2/dt_t)^2; the lumped masses use the scaled
densities.

Pins (tests/test_oracle_cfl.py): the global generalized eigenvalue never
exceeds the bound (also with scaled masses); the undamped scheme stays
bounded at 0.99 * 2/omega_glob and diverges at 1.05 * 2/omega_glob; mass
scaling leaves unscaled elements exactly alone and makes the scaled bound
(2/dt_t)^2.
"""
from __future__ import annotations

import numpy as np


def element_lambda_max(khat: np.ndarray) -> np.ndarray:
    """Largest eigenvalue of each symmetric 9x9 Khat_e."""
    return np.linalg.eigvalsh(khat)[:, -1]


def element_omega2(khat: np.ndarray, area: np.ndarray, eh: np.ndarray, h: np.ndarray, rho: float) -> np.ndarray:
    """3 E_{e,s} lambda_max(Khat_e) / (rho A_e) [n_el, S]."""
    lam = element_lambda_max(khat)
    return 3.0 * (eh / h) * (lam / (rho * area))[:, None]


def mass_scale_factors(khat, area, eh, h, rho, dt_target: float) -> np.ndarray:
    """Density factors f_{e,s} = max(1, omega2_e,s dt_target^2 / 4)."""
    return np.maximum(1.0, element_omega2(khat, area, eh, h, rho) * (dt_target * dt_target / 4.0))


def omega2_bound(khat: np.ndarray, area: np.ndarray, eh: np.ndarray, h: np.ndarray, rho: float,
                 scale: np.ndarray = None) -> float:
    w2 = element_omega2(khat, area, eh, h, rho)
    if scale is not None:
        w2 = w2 / scale
    return float(np.max(w2))


def stable_dt(khat, area, eh, h, rho, safety: float = 0.9, scale: np.ndarray = None) -> float:
    return safety * 2.0 / np.sqrt(omega2_bound(khat, area, eh, h, rho, scale))
