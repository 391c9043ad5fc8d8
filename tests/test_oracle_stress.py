"""Pins of the oracle's wall stresses in the cylindrical frame."""
import math

import numpy as np
import scipy.sparse.linalg as spla

from oracle import assembly, element, stress
from paper_2101_09059_amd import inputs


def _flat_patch():
    xs, ys = np.meshgrid(np.linspace(0, 1, 5), np.linspace(0, 2, 6))
    xyz = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size)], 1)
    tri = []
    for j in range(5):
        for i in range(4):
            a = j * 5 + i
            tri += [(a, a + 1, a + 6), (a, a + 6, a + 5)]
    return xyz, np.array(tri, dtype=np.int32)


def test_rigid_motions_give_zero_stress():
    m = inputs.cylinder(1.0, 4.0, 16, 7)
    rng = np.random.default_rng(1)
    E = 7e6 * np.exp(0.2 * rng.standard_normal(m.n_el))
    axial = np.tile([0.0, 0.0, 1.0], (m.n_el, 1))
    t = rng.standard_normal(3)
    u = np.tile(t, m.n_nodes)
    s = stress.cylindrical_stress(m.xyz, m.tri, u, E, 0.49, 5.0 / 6.0, axial)
    assert np.max(np.abs(s)) < 1e-8 * 7e6 * np.linalg.norm(t)
    w = rng.standard_normal(3) * 1e-3
    u = np.cross(w, m.xyz).reshape(-1)
    s0 = stress.cylindrical_stress(m.xyz, m.tri, u, E, 0.49, 0.0, axial)
    assert np.max(np.abs(s0)) < 1e-8 * 7e6 * np.linalg.norm(w)


def test_homogeneous_gradient_on_a_flat_patch():
    """u = G x on a patch in the xy-plane (normals +z): eps_xx = G00,
    eps_yy = G11, gamma_xy = G01 + G10, du_z/dx = G20, du_z/dy = G21; with the
    axis along y, theta = z x y = -x, so sigma_thth = sigma_xx,
    sigma_zz = sigma_yy, sigma_thz = -tau_xy, sigma_rz = tau_yz."""
    xyz, tri = _flat_patch()
    nu, k, E0 = 0.3, 5.0 / 6.0, 2.0e6
    G = np.array([[1.0, 0.3, 0.0], [-0.2, 0.5, 0.0], [0.7, -0.4, 0.0]]) * 1e-3
    u = (xyz @ G.T).reshape(-1)
    E = np.full(tri.shape[0], E0)
    axial = np.tile([0.0, 1.0, 0.0], (tri.shape[0], 1))
    s = stress.cylindrical_stress(xyz, tri, u, E, nu, k, axial)
    exx, eyy, gxy, gxz, gyz = G[0, 0], G[1, 1], G[0, 1] + G[1, 0], G[2, 0], G[2, 1]
    c = E0 / (1 - nu * nu)
    sxx = c * (exx + nu * eyy)
    syy = c * (nu * exx + eyy)
    txy = c * 0.5 * (1 - nu) * gxy
    tyz = c * 0.5 * k * (1 - nu) * gyz
    expect = np.array([sxx, syy, -txy, tyz])
    assert np.allclose(s, expect[None, :], rtol=1e-12, atol=1e-9 * abs(sxx))


def test_laplace_hoop_stress_middle_ring():
    """Static pressurised clamped cylinder, homogeneous E h: the hoop stress
    of the elements at mid-length times the thickness equals the faceted
    hoop resultant p R cos(pi / n) to 1e-3."""
    nu, E, h, p, R = 0.49, 7e6, 0.1, 1.33e5, 1.0
    m = inputs.cylinder(R, 10.0, 40, 20)
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, nu, 5.0 / 6.0)
    K = assembly.assemble_stiffness(m.tri, kh, np.full(m.n_el, E * h), m.n_nodes)
    F = inputs.traction_load(m, p).reshape(-1)
    free = ~m.fixed.reshape(-1).astype(bool)
    u = np.zeros(m.n_dof)
    u[free] = spla.spsolve(K[free][:, free].tocsc(), F[free])
    axial = np.tile([0.0, 0.0, 1.0], (m.n_el, 1))
    s = stress.cylindrical_stress(m.xyz, m.tri, u, np.full(m.n_el, E), nu, 5.0 / 6.0, axial)
    zc = m.xyz[m.tri, 2].mean(axis=1)
    mid = np.abs(zc - 5.0) < 0.3
    target = p * R * math.cos(math.pi / m.n_theta)
    assert np.max(np.abs(s[mid, 0] * h / target - 1.0)) < 1e-3


def test_invariant_under_rigid_rotation():
    m = inputs.curved_tube(12, 9)
    rng = np.random.default_rng(3)
    E = 7e6 * np.exp(0.2 * rng.standard_normal(m.n_el))
    u = rng.standard_normal(m.n_dof) * 1e-3
    axial = rng.standard_normal((m.n_el, 3))
    axial /= np.linalg.norm(axial, axis=1, keepdims=True)
    s0 = stress.cylindrical_stress(m.xyz, m.tri, u, E, 0.49, 5.0 / 6.0, axial)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    s1 = stress.cylindrical_stress(m.xyz @ Q.T, m.tri, (u.reshape(-1, 3) @ Q.T).reshape(-1), E, 0.49, 5.0 / 6.0,
                                   axial @ Q.T)
    assert np.allclose(s1, s0, rtol=1e-10, atol=1e-10 * np.abs(s0).max())


def test_bands_are_numpy_percentiles():
    v = np.random.default_rng(4).standard_normal((7, 33))
    mean, lo, hi = stress.ensemble_bands(v, 0.05, 0.95)
    srt = np.sort(v, axis=1)
    pos = 0.05 * 32
    i = int(math.floor(pos))
    assert np.allclose(lo, srt[:, i] + (pos - i) * (srt[:, i + 1] - srt[:, i]))
    assert np.allclose(mean, v.sum(1) / 33)
    assert np.all(hi >= lo)
