"""Laplace-law pin: homogeneous clamped cylinder under internal pressure.

Away from the clamped ends the hoop resultant of the faceted cylinder is
fixed by statics alone: each facet of the n-gon carries p * chord, half to
each node along the facet normal, so N_theta = p R cos(pi / n).  The radial
displacement lies between the plane-strain and the free-end thin-tube values
(1 - nu^2) p R^2 / (E h) and p R^2 / (E h).
"""
import math

import numpy as np
import scipy.sparse.linalg as spla

from oracle import assembly, element
from paper_2101_09059_amd import inputs


def test_laplace_hoop_resultant_middle_ring():
    nu, E, h, p, R = 0.49, 7e6, 0.1, 1.33e5, 1.0
    m = inputs.cylinder(R, 10.0, 40, 20)
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, nu, 5.0 / 6.0)
    K = assembly.assemble_stiffness(m.tri, kh, np.full(m.n_el, E * h), m.n_nodes)
    F = inputs.traction_load(m, p).reshape(-1)
    free = ~m.fixed.reshape(-1).astype(bool)
    u = np.zeros(m.n_dof)
    u[free] = spla.spsolve(K[free][:, free].tocsc(), F[free])
    U = u.reshape(-1, 3)
    nt, nz = m.n_theta, m.n_z
    ring = np.arange(nt) + (nz // 2) * nt
    x0 = m.xyz[ring]
    x1 = x0 + U[ring]
    c0 = np.linalg.norm(np.roll(x0, -1, 0) - x0, axis=1)
    c1 = np.linalg.norm(np.roll(x1, -1, 0) - x1, axis=1)
    eps_t = (c1 - c0) / c0
    dz = m.length / (nz - 1)
    eps_z = (U[ring + nt, 2] - U[ring - nt, 2]) / (2 * dz)
    n_theta_res = E * h / (1 - nu * nu) * (eps_t + nu * eps_z)
    target = p * R * math.cos(math.pi / nt)
    assert np.max(np.abs(n_theta_res / target - 1.0)) < 1e-3
    w = np.sum(U[ring] * m.radial[ring], axis=1).mean()
    assert (1 - nu * nu) * p * R * R / (E * h) < w < p * R * R / (E * h)
