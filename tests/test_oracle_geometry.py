"""Pins for the oracle's geometry update with selective stiffness refresh
(Sec. 2.3): invariances of the rebuilt matrix, the patch test on a
stretched geometry, and the refresh schedule against chained plain runs."""
import numpy as np
import pytest

from oracle import assembly, element, geometry, stepper
from tests._cases import small_case

NU, KS = 0.49, 5.0 / 6.0


def _mesh_matrix(cs, u):
    return geometry.deformed_stiffness(cs.mesh.xyz, cs.mesh.tri, u, cs.eh[:, 0], NU, KS).toarray()


def test_rigid_motions_and_scaling():
    cs = small_case(10, 5, 1, seed=3)
    x = cs.mesh.xyz
    K0 = _mesh_matrix(cs, np.zeros(x.size))
    scale = np.abs(K0).max()
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    # rigid rotation: K(Q x) = diag(Q) K(x) diag(Q)^T
    Kr = _mesh_matrix(cs, (x @ Q.T - x).ravel())
    T = np.kron(np.eye(x.shape[0]), Q)
    assert np.max(np.abs(Kr - T @ K0 @ T.T)) <= 1e-12 * scale
    # translation and uniform scaling leave the linear triangle's matrix alone
    Kt = _mesh_matrix(cs, np.tile([0.3, -1.2, 2.5], x.shape[0]))
    assert np.max(np.abs(Kt - K0)) <= 1e-12 * scale
    Ks = _mesh_matrix(cs, (1.7 * x - x).ravel())
    assert np.max(np.abs(Ks - K0)) <= 1e-12 * scale
    # a shear of the geometry does change it
    Sh = np.array([[1.0, 0.0, 0.4], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    Kh = _mesh_matrix(cs, (x @ Sh.T - x).ravel())
    assert np.max(np.abs(Kh - K0)) > 1e-3 * scale


@pytest.mark.parametrize("lam", [1.0, 1.6])
def test_patch_test_on_stretched_plate(lam):
    """Flat 1 x 1 plate stretched to lam x 1: a field linear in the moved
    coordinates has strain energy (area lam) x 1/2 eps^T C eps."""
    n = 6
    g = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(g, g)
    xyz = np.stack([X.ravel(), Y.ravel(), np.zeros(n * n)], 1)
    tri = []
    for j in range(n - 1):
        for i in range(n - 1):
            a = j * n + i
            tri += [(a, a + 1, a + n + 1), (a, a + n + 1, a + n)]
    tri = np.array(tri, dtype=np.int32)
    moved = xyz * np.array([lam, 1.0, 1.0])
    K = geometry.deformed_stiffness(xyz, tri, (moved - xyz).ravel(), np.ones(len(tri)), NU, KS)
    G = np.array([[0.3, -0.2, 0.0], [0.5, 0.1, 0.0], [0.7, -0.4, 0.0]])  # du_i/dx'_j, plate in z = 0
    u = (moved @ G.T).ravel()
    eps = np.array([G[0, 0], G[1, 1], G[0, 1] + G[1, 0], G[2, 0], G[2, 1]])
    C = element.constitutive_unit(NU, KS)
    expect = 0.5 * lam * eps @ C @ eps
    assert abs(0.5 * u @ (K @ u) - expect) <= 1e-12 * expect


def _setup(load):
    cs = small_case(12, 6, 1, seed=5)
    m = cs.mesh
    F = load * cs.F.reshape(-1)
    fx = m.fixed.reshape(-1).astype(bool)
    mass = assembly.lumped_mass(m.tri, cs.area, cs.h[:, 0], 1.0, m.n_nodes)
    K0 = assembly.assemble_stiffness(m.tri, cs.khat, cs.eh[:, 0], m.n_nodes)
    g = lambda t: stepper.load_factor("sine", t, T_ramp=20 * cs.dt)
    K_at = lambda u: geometry.deformed_stiffness(m.xyz, m.tri, u, cs.eh[:, 0], NU, KS)
    return cs, F, fx, mass, K0, g, K_at


def test_refresh_schedule_equals_chained_plain_runs():
    cs, F, fx, mass, K0, g, K_at = _setup(0.3)
    every, seg = 5, 4
    ref = stepper.run_sample(K0, mass, F, fx, cs.dt, every * seg, 50.0, g, K_at=K_at, every=every)
    # chained: `every` plain steps with the force R_b + K (u - u_b), then
    # R_b += K (u - u_b), u_b = u, K = K(x + u), and again
    K, u, up = K0, None, None
    Rb, ub = np.zeros(F.size), np.zeros(F.size)
    for k in range(seg):
        t0 = k * every * cs.dt
        r = stepper.run_sample(K, mass, F, fx, cs.dt, every, 50.0, lambda t, t0=t0: g(t + t0),
                               u0=u, u_prev=up, R_base=Rb, u_base=ub)
        u, up = r["u"], r["u_prev"]
        Rb, ub = Rb + K @ (u - ub), u.copy()
        K = K_at(u)
    assert np.max(np.abs(ref["u"] - u)) <= 1e-14 * np.max(np.abs(u))
    plain = stepper.run_sample(K0, mass, F, fx, cs.dt, every * seg, 50.0, g)
    # the refresh matters at this load, and never firing it is the plain run
    assert np.linalg.norm(ref["u"] - plain["u"]) > 1e-6 * np.linalg.norm(plain["u"])
    never = stepper.run_sample(K0, mass, F, fx, cs.dt, every * seg, 50.0, g, K_at=K_at, every=10 * every * seg)
    assert np.array_equal(never["u"], plain["u"])


def test_vanishing_load_gives_the_linear_run():
    """The refresh changes the force by O(|u| / element size): scaling the
    load down by 1e4 brings the refreshed run to the linear one."""
    diffs = []
    for load in (1.0, 1e-4):
        cs, F, fx, mass, K0, g, K_at = _setup(load)
        ref = stepper.run_sample(K0, mass, F, fx, cs.dt, 200, 50.0, g, K_at=K_at, every=3)
        plain = stepper.run_sample(K0, mass, F, fx, cs.dt, 200, 50.0, g)
        diffs.append(np.linalg.norm(ref["u"] - plain["u"]) / np.linalg.norm(plain["u"]))
    assert diffs[0] > 1e-3
    assert diffs[1] < 1e-3 * diffs[0]


@pytest.mark.parametrize("k", [1, 4, 16])
def test_stretch_in_refreshed_increments_carries_the_sum_of_edge_tractions(k):
    """Flat 1 x 1 plate (z = 0, unit E h) stretched along x from 1 to 1.6 in
    k equal increments, the matrix rebuilt on the stretched plate after each.
    Increment j is a homogeneous strain eps_j = dlam / lam_{j-1} of the plate
    as stretched before it (width lam_{j-1}), so its nodal forces are the
    edge tractions of sigma = C eps_j: zero inside, sigma_xx eps_j / (1 -
    nu^2) on the right edge (height 1), nu eps_j / (1 - nu^2) lam_{j-1} on
    the top edge.  The carried force is the sum over the increments; the
    total form K_{k-1} u_k would put (lam_k - 1) / lam_{k-1} on the edge."""
    n = 7
    g = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(g, g)
    xyz = np.stack([X.ravel(), Y.ravel(), np.zeros(n * n)], 1)
    tri = []
    for j in range(n - 1):
        for i in range(n - 1):
            a = j * n + i
            if (i + j) % 2:
                tri += [(a, a + 1, a + n + 1), (a, a + n + 1, a + n)]
            else:
                tri += [(a, a + 1, a + n), (a + 1, a + n + 1, a + n)]
    tri = np.array(tri, dtype=np.int32)
    ones = np.ones(len(tri))
    K_at = lambda u: geometry.deformed_stiffness(xyz, tri, u, ones, NU, KS)
    lam = np.linspace(1.0, 1.6, k + 1)
    path = [((l - 1.0) * xyz * np.array([1.0, 0.0, 0.0])).ravel() for l in lam]
    force = geometry.IncrementalForce(K_at(path[0]), K_at)
    for j in range(1, k):
        force.refresh(path[j])
    R = force.force(path[k]).reshape(-1, 3)
    eps = np.diff(lam) / lam[:-1]
    fx_right = np.sum(eps) / (1.0 - NU * NU)
    fy_top = np.sum(NU * eps * lam[:-1]) / (1.0 - NU * NU)
    right = np.isclose(xyz[:, 0], 1.0)
    top = np.isclose(xyz[:, 1], 1.0)
    inner = ~(right | top | np.isclose(xyz[:, 0], 0.0) | np.isclose(xyz[:, 1], 0.0))
    scale = fx_right
    assert abs(R[right, 0].sum() - fx_right) <= 1e-12 * scale
    assert abs(R[top, 1].sum() - fy_top) <= 1e-12 * scale
    # each right-edge node carries its share of the edge (corners half)
    share = np.where(np.isclose(xyz[right, 1], 0.0) | np.isclose(xyz[right, 1], 1.0), 0.5, 1.0) / (n - 1)
    assert np.max(np.abs(R[right, 0] - fx_right * share)) <= 1e-12 * scale
    assert np.max(np.abs(R[inner])) <= 1e-12 * scale
    assert np.max(np.abs(R[:, 2])) <= 1e-12 * scale
    if k > 1:
        total = (lam[-1] - 1.0) / lam[-2] / (1.0 - NU * NU)
        assert abs(total - fx_right) > 1e-2 * fx_right
