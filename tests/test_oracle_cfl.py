"""Pins for the element-eigenvalue step bound."""
import math

import numpy as np
import scipy.linalg as sla

from oracle import assembly, cfl, stepper, element, matern
from paper_2101_09059_amd import inputs
from tests._mesh_helpers import tiny_case, free_system


def _global_omega2(m, kh, A, eh_col, h_col, clamp=False):
    K, mn, free = free_system(m, kh, A, eh_col, h_col)
    Kd = K.toarray()
    md = np.repeat(mn, 3)
    if clamp:
        Kd = Kd[np.ix_(free, free)]
        md = md[free]
    s = 1.0 / np.sqrt(md)
    return float(np.linalg.eigvalsh(s[:, None] * Kd * s[None, :])[-1])


def test_global_eigenvalue_below_element_bound_c1_mesh():
    m = inputs.cylinder(1.0, 10.0, 40, 20)
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, 0.49, 5.0 / 6.0)
    eh, h = matern.lognormal_fields(m.xyz, m.tri, 2, seed=1)
    bound = cfl.omega2_bound(kh, A, eh, h, 1.0)
    for s in range(2):
        w2 = _global_omega2(m, kh, A, eh[:, s], h[:, s])
        assert w2 <= bound * (1 + 1e-12)
        assert w2 >= 0.3 * bound      # the bound is not vacuous on this mesh
    # homogeneous wall: dt = 0.9 * 2 / omega_hat, with omega_hat independent of h
    e1 = np.full((m.n_el, 1), 7e6 * 0.1)
    dt = cfl.stable_dt(kh, A, e1, np.full((m.n_el, 1), 0.1), 1.0, 0.9)
    dt2 = cfl.stable_dt(kh, A, 2 * e1, np.full((m.n_el, 1), 0.2), 1.0, 0.9)
    assert abs(dt - dt2) <= 1e-15 * dt


def test_stability_threshold():
    m, kh, A, eh, h = tiny_case()
    K, mn, free = free_system(m, kh, A, eh[:, 0], h[:, 0])
    w = math.sqrt(_global_omega2(m, kh, A, eh[:, 0], h[:, 0], clamp=True))
    rng = np.random.default_rng(3)
    u0 = np.where(free, rng.normal(size=m.n_dof), 0.0)
    ok = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, 0.99 * 2 / w, 3000, 0.0, lambda t: 0.0, u0=u0)
    assert np.linalg.norm(ok["u"]) < 50 * np.linalg.norm(u0)
    bad = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, 1.05 * 2 / w, 300, 0.0, lambda t: 0.0, u0=u0)
    assert np.linalg.norm(bad["u"]) > 1e6 * np.linalg.norm(u0)


def test_mass_scaling():
    """Scaling to a target step 1.5x the unscaled one: unscaled elements keep
    factor 1 exactly, the scaled bound is (2/dt_t)^2, the global eigenvalue
    of the pencil with the scaled masses stays below it, and the undamped
    scheme is stable at 0.99 dt_t."""
    m = inputs.cylinder(1.0, 10.0, 40, 20)
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, 0.49, 5.0 / 6.0)
    eh, h = matern.lognormal_fields(m.xyz, m.tri, 2, seed=1)
    dt0 = cfl.stable_dt(kh, A, eh, h, 1.0, 1.0)
    dt_t = 1.5 * dt0
    f = cfl.mass_scale_factors(kh, A, eh, h, 1.0, dt_t)
    w2 = cfl.element_omega2(kh, A, eh, h, 1.0)
    assert np.all(f[w2 * dt_t * dt_t <= 4.0] == 1.0)
    assert np.any(f > 1.0)
    bound = cfl.omega2_bound(kh, A, eh, h, 1.0, f)
    assert abs(bound * dt_t * dt_t / 4.0 - 1.0) < 1e-12
    assert cfl.stable_dt(kh, A, eh, h, 1.0, 1.0, f) >= dt_t * (1 - 1e-12)
    # a target below the current step changes nothing
    assert np.all(cfl.mass_scale_factors(kh, A, eh, h, 1.0, 0.5 * dt0) == 1.0)
    for s in range(2):
        K = assembly.assemble_stiffness(m.tri, kh, eh[:, s], m.n_nodes)
        mn = assembly.lumped_mass(m.tri, A, h[:, s], 1.0, m.n_nodes, f[:, s])
        mn0 = assembly.lumped_mass(m.tri, A, h[:, s], 1.0, m.n_nodes)
        assert np.all(mn >= mn0) and mn.sum() > mn0.sum()
        md = np.repeat(mn, 3)
        sc = 1.0 / np.sqrt(md)
        wg = float(np.linalg.eigvalsh(sc[:, None] * K.toarray() * sc[None, :])[-1])
        assert wg <= bound * (1 + 1e-12)
    free = ~m.fixed.reshape(-1).astype(bool)
    rng = np.random.default_rng(5)
    u0 = np.where(free, rng.normal(size=m.n_dof), 0.0)
    K = assembly.assemble_stiffness(m.tri, kh, eh[:, 0], m.n_nodes)
    mn = assembly.lumped_mass(m.tri, A, h[:, 0], 1.0, m.n_nodes, f[:, 0])
    ok = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, 0.99 * dt_t, 3000, 0.0, lambda t: 0.0, u0=u0)
    assert np.linalg.norm(ok["u"]) < 50 * np.linalg.norm(u0)
