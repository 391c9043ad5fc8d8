"""Pins for the oracle's shell element (Sec. 2.2.1).

Independent checks: eigen-structure, rigid-body null spaces, frame
invariance, and energies of linear displacement fields compared with the
textbook plane-stress moduli (uniaxial stress E, in-plane shear
G = E / (2 (1 + nu)), transverse shear k G).
"""
import numpy as np
import pytest

from oracle import element

NU = 0.49


def _tri(rng):
    p = rng.normal(size=(3, 3))
    return p


def _khat(p, k):
    kh, A, n = element.reference_stiffness(p, np.array([[0, 1, 2]]), NU, k)
    return kh[0], A[0], n[0]


@pytest.mark.parametrize("k", [5.0 / 6.0, 0.0])
def test_symmetric_psd_rank(k):
    rng = np.random.default_rng(0)
    for _ in range(20):
        kh, A, _ = _khat(_tri(rng), k)
        scale = np.max(np.abs(kh))
        assert np.max(np.abs(kh - kh.T)) <= 1e-13 * scale
        ev = np.linalg.eigvalsh(kh)
        assert ev[0] >= -1e-13 * ev[-1]
        rank = int(np.sum(ev > 1e-10 * ev[-1]))
        assert rank == (5 if k > 0 else 3)


@pytest.mark.parametrize("k", [5.0 / 6.0, 0.0])
def test_translation_null_space(k):
    rng = np.random.default_rng(1)
    for _ in range(20):
        kh, _, _ = _khat(_tri(rng), k)
        for c in range(3):
            t = np.zeros(9)
            t[c::3] = 1.0
            assert np.linalg.norm(kh @ t) <= 1e-13 * np.linalg.norm(kh)


def test_rotation_null_space_membrane_only():
    # infinitesimal rotation u_j = w x p_j: zero force at k = 0; at k = 5/6 the
    # transverse-shear rows penalise out-of-plane rotation
    rng = np.random.default_rng(2)
    for _ in range(20):
        p = _tri(rng)
        w = rng.normal(size=3)
        u = np.cross(w, p).reshape(-1)
        kh0, _, _ = _khat(p, 0.0)
        assert np.linalg.norm(kh0 @ u) <= 1e-13 * np.linalg.norm(kh0) * np.linalg.norm(u)
    p = _tri(rng)
    khk, _, n = _khat(p, 5.0 / 6.0)
    w = np.cross(n, [1.0, 0.0, 0.0])       # in-plane axis -> tilts the element
    u = np.cross(w, p).reshape(-1)
    assert np.linalg.norm(khk @ u) > 1e-3 * np.linalg.norm(khk) * np.linalg.norm(u)


def test_cyclic_relabelling_and_rigid_rotation():
    rng = np.random.default_rng(3)
    for _ in range(10):
        p = _tri(rng)
        kh, A, _ = _khat(p, 5.0 / 6.0)
        # relabel (p2, p3, p1)
        kp, Ap, _ = _khat(p[[1, 2, 0]], 5.0 / 6.0)
        perm = np.r_[3:9, 0:3]
        assert np.allclose(kp, kh[np.ix_(perm, perm)], rtol=0, atol=1e-13 * np.abs(kh).max())
        assert abs(Ap - A) <= 1e-14 * A
        # rotate the triangle rigidly by Q: Khat' = diag(Q) Khat diag(Q)^T
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] *= -1
        kr, _, _ = _khat(p @ Q.T + rng.normal(size=3), 5.0 / 6.0)
        T = np.kron(np.eye(3), Q)
        assert np.allclose(kr, T @ kh @ T.T, rtol=0, atol=1e-13 * np.abs(kh).max())


def test_patch_energies_planar_triangle():
    # triangle in the xy plane with p2 on the +x axis: the local frame is the
    # global one, so a linear field's strains are known in closed form
    E = 1.0
    G = E / (2.0 * (1.0 + NU))
    k = 5.0 / 6.0
    p = np.array([[0.0, 0.0, 0.0], [1.3, 0.0, 0.0], [0.4, 0.9, 0.0]])
    kh, A, n = _khat(p, k)
    assert np.allclose(n, [0, 0, 1])
    assert abs(A - 0.5 * 1.3 * 0.9) < 1e-15

    def field(fx, fy, fz):
        return np.array([[fx(q), fy(q), fz(q)] for q in p]).reshape(-1)

    # uniaxial stress along x: eps_xx = e, eps_yy = -nu e  ->  energy 1/2 E e^2 A
    e = 1e-3
    u = field(lambda q: e * q[0] + 0.2, lambda q: -NU * e * q[1] - 0.1, lambda q: 0.3)
    assert np.isclose(0.5 * u @ kh @ u, 0.5 * E * e * e * A, rtol=1e-13)
    # same along y
    u = field(lambda q: -NU * e * q[0], lambda q: e * q[1], lambda q: 0.0)
    assert np.isclose(0.5 * u @ kh @ u, 0.5 * E * e * e * A, rtol=1e-13)
    # in-plane engineering shear gamma: u_x = gamma y  -> 1/2 G gamma^2 A
    gam = 2e-3
    u = field(lambda q: gam * q[1], lambda q: 0.0, lambda q: 0.0)
    assert np.isclose(0.5 * u @ kh @ u, 0.5 * G * gam * gam * A, rtol=1e-13)
    # transverse shear: u_z = a x + b y  ->  1/2 k G (a^2 + b^2) A
    a, b = 1e-3, -2e-3
    u = field(lambda q: 0.0, lambda q: 0.0, lambda q: a * q[0] + b * q[1])
    assert np.isclose(0.5 * u @ kh @ u, 0.5 * k * G * (a * a + b * b) * A, rtol=1e-13)
    # equal biaxial strain e: plane-stress energy density E e^2 / (1 - nu)
    u = field(lambda q: e * q[0], lambda q: e * q[1], lambda q: 0.0)
    assert np.isclose(0.5 * u @ kh @ u, E * e * e / (1.0 - NU) * A, rtol=1e-13)
