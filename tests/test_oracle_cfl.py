"""Pins for the element-eigenvalue step bound."""
import math

import numpy as np
import scipy.linalg as sla

from oracle import cfl, stepper, element, matern
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
