"""Wall stresses in the local cylindrical frame and their ensemble bands --
oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Per element (Sec. 2.2.1): local strains eps = B u_loc (u_loc the element's
nodal displacements in its local frame), local stresses
sigma_loc = C eps = (sigma_xx, sigma_yy, tau_xy, tau_xz, tau_yz) with
C = E/(1-nu^2) [[1,nu],[nu,1]] (+) (1-nu)/2 (+) k(1-nu)/2 (+) k(1-nu)/2 and
sigma_zz = 0, i.e. the local tensor [[sxx, txy, txz], [txy, syy, tyz],
[txz, tyz, 0]], rotated to the global frame (R^T S R, R's rows the local
axes).  The cylindrical frame of Sec. 2.3 (fluid-structure coupling): r the
element's unit normal, z the centreline tangent, theta = r x z.  The paper
does not say what to do when the tangent is not in the element's plane (a
tapered or curved tube); here z is the tangent with its normal component
removed, normalised, so (r, theta, z) is orthonormal.  Outputs per element
and sample: sigma_thth, sigma_zz, sigma_thz, sigma_rz.

Ensemble bands: mean over samples and the p-quantiles by linear
interpolation between order statistics at position p (S - 1) (numpy's
default percentile).

Pins (tests/test_oracle_stress.py): zero stress under rigid translations
(and infinitesimal rotations at k = 0); a homogeneous displacement gradient
on a flat patch against the constitutive law written out by hand; the Laplace
law sigma_thth h = p R cos(pi / n) at the middle of a pressurised clamped
cylinder; invariance under a rigid rotation of mesh, displacements and axes.
"""
from __future__ import annotations

import numpy as np

from . import element

COMPONENTS = ("theta_theta", "z_z", "theta_z", "r_z")


def cylindrical_stress(xyz: np.ndarray, tri: np.ndarray, u: np.ndarray, E: np.ndarray, nu: float,
                       shear_k: float, axial: np.ndarray) -> np.ndarray:
    """u [n_dof] (one sample, global components), E [n_el], axial [n_el, 3]
    centreline tangents.  Returns [n_el, 4] in COMPONENTS order."""
    p1, p2, p3 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    Rm, x, y = element.local_frames(p1, p2, p3)
    A = element.areas(x, y)
    B = element.strain_matrix(x, y, A)
    ue = u.reshape(-1, 3)[tri]                                   # [m, 3 nodes, 3]
    ul = np.einsum("mij,mnj->mni", Rm, ue).reshape(-1, 9)        # local components
    eps = np.einsum("mij,mj->mi", B, ul)
    sig = E[:, None] * (eps @ element.constitutive_unit(nu, shear_k).T)
    sxx, syy, txy, txz, tyz = sig.T
    S = np.zeros((tri.shape[0], 3, 3))
    S[:, 0, 0], S[:, 1, 1] = sxx, syy
    S[:, 0, 1] = S[:, 1, 0] = txy
    S[:, 0, 2] = S[:, 2, 0] = txz
    S[:, 1, 2] = S[:, 2, 1] = tyz
    Sg = np.einsum("mai,mab,mbj->mij", Rm, S, Rm)                # R^T S R
    er = Rm[:, 2, :]
    z = axial - np.sum(axial * er, axis=1, keepdims=True) * er
    ez = z / np.linalg.norm(z, axis=1, keepdims=True)
    et = np.cross(er, ez)
    q = lambda a, b: np.einsum("mi,mij,mj->m", a, Sg, b)
    return np.stack([q(et, et), q(ez, ez), q(et, ez), q(er, ez)], axis=1)


def ensemble_bands(values: np.ndarray, p_lo: float, p_hi: float):
    """values [n_el, S] -> mean, p_lo- and p_hi-quantiles [n_el]."""
    return values.mean(axis=1), np.percentile(values, 100 * p_lo, axis=1), np.percentile(values, 100 * p_hi, axis=1)
