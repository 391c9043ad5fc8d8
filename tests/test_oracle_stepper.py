"""Pins for the oracle's central-difference stepper (Sec. 2.3, eq. dynamicsCD)."""
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import stepper
from tests._mesh_helpers import tiny_case, free_system


def _modes(m, kh, A, eh, h):
    K, mn, free = free_system(m, kh, A, eh[:, 0], h[:, 0])
    Kd = K.toarray()[np.ix_(free, free)]
    Md = np.repeat(mn, 3)[free]
    w2, phi = sla.eigh(Kd, np.diag(Md))
    return K, mn, free, w2, phi


def _embed(free, x):
    u = np.zeros(free.size)
    u[free] = x
    return u


def test_single_mode_closed_form_undamped():
    m, kh, A, eh, h = tiny_case()
    K, mn, free, w2, phi = _modes(m, kh, A, eh, h)
    dt = 0.8 * 2.0 / math.sqrt(w2[-1])
    for idx in (0, len(w2) // 2, len(w2) - 1):
        Om2 = w2[idx] * dt * dt
        theta = math.acos(1.0 - 0.5 * Om2)
        ph = _embed(free, phi[:, idx])
        n = 2000
        r = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, dt, n, 0.0, lambda t: 0.0,
                               u0=ph, u_prev=ph * math.cos(theta))
        exact = ph * math.cos(n * theta)
        assert np.linalg.norm(r["u"] - exact) <= 1e-11 * np.linalg.norm(ph)


def test_single_mode_closed_form_damped():
    m, kh, A, eh, h = tiny_case()
    K, mn, free, w2, phi = _modes(m, kh, A, eh, h)
    dt = 0.8 * 2.0 / math.sqrt(w2[-1])
    alpha = 300.0
    a = 0.5 * alpha * dt
    for idx in (0, len(w2) - 1):
        Om2 = w2[idx] * dt * dt
        lam = np.roots([1.0 + a, -(2.0 - Om2), 1.0 - a]).astype(complex)
        beta = 0.7
        # u_0 = phi, u_{-1} = beta phi  ->  u_n = phi (c1 l1^n + c2 l2^n)
        M = np.array([[1.0, 1.0], [1.0 / lam[0], 1.0 / lam[1]]])
        c = np.linalg.solve(M, np.array([1.0, beta], dtype=complex))
        ph = _embed(free, phi[:, idx])
        n = 500
        r = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, dt, n, alpha, lambda t: 0.0,
                               u0=ph, u_prev=beta * ph)
        amp = (c[0] * lam[0] ** n + c[1] * lam[1] ** n).real
        assert np.linalg.norm(r["u"] - amp * ph) <= 1e-11 * np.linalg.norm(ph)


def test_energy_conserved_undamped_unforced():
    m, kh, A, eh, h = tiny_case()
    K, mn, free, w2, phi = _modes(m, kh, A, eh, h)
    dt = 0.9 * 2.0 / math.sqrt(w2[-1])
    rng = np.random.default_rng(7)
    u0 = _embed(free, rng.normal(size=free.sum()))
    r = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, dt, 2000, 0.0, lambda t: 0.0,
                           u0=u0, energy_every=1)
    E = np.array([e for _, e in r["energy"]])
    assert np.max(np.abs(E - E[0])) <= 1e-12 * abs(E[0])


def test_energy_balance_constant_force_and_damped_decay():
    m, kh, A, eh, h = tiny_case()
    K, mn, free, w2, phi = _modes(m, kh, A, eh, h)
    dt = 0.9 * 2.0 / math.sqrt(w2[-1])
    rng = np.random.default_rng(8)
    F = rng.normal(size=m.n_dof) * 1e3
    n = 600
    r = stepper.run_sample(K, mn, F, ~free, dt, n, 0.0, lambda t: 1.0, energy_every=1,
                           checkpoints=range(n + 1))
    Ff = np.where(free, F, 0.0)
    cps = r["checkpoints"]
    H = np.array([e - 0.5 * Ff @ (cps[k + 1] + cps[k]) for k, e in r["energy"]])
    assert np.max(np.abs(H - H[0])) <= 1e-11 * np.max(np.abs([e for _, e in r["energy"]]))
    # damped and unforced: the discrete energy never increases
    u0 = _embed(free, rng.normal(size=free.sum()))
    r = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, dt, n, 40.0, lambda t: 0.0,
                           u0=u0, energy_every=1)
    E = np.array([e for _, e in r["energy"]])
    assert np.all(np.diff(E) <= 1e-12 * E[0])
    assert E[-1] < 0.9 * E[0]


def test_viscous_force_discrete_energy_balance():
    """With the explicit viscous force f_v = -c_d (u_n - u_{n-1}) / dt and no
    other force or damping, multiplying the update by (u_{n+1} - u_{n-1}) / 2
    gives E_{n+1/2} - E_{n-1/2} = -c_d dt / 2 v_{n-1/2} . (v_{n+1/2} + v_{n-1/2})
    exactly (v_{n+1/2} = (u_{n+1} - u_n) / dt); the energy then decays."""
    m, kh, A, eh, h = tiny_case()
    K, mn, free, w2, phi = _modes(m, kh, A, eh, h)
    dt = 0.9 * 2.0 / math.sqrt(w2[-1])
    c_d = 0.05 * mn.min() / dt
    rng = np.random.default_rng(10)
    u0 = _embed(free, rng.normal(size=free.sum()))
    n = 400
    r = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, dt, n, 0.0, lambda t: 0.0, u0=u0,
                           energy_every=1, checkpoints=range(n + 1), c_d=c_d)
    E = np.array([e for _, e in r["energy"]])
    cps = r["checkpoints"]
    v = [(cps[k + 1] - cps[k]) / dt for k in range(n)]
    pred = np.array([-0.5 * c_d * dt * v[k - 1] @ (v[k] + v[k - 1]) for k in range(1, n)])
    assert np.max(np.abs(np.diff(E) - pred)) <= 1e-10 * E[0]
    assert np.all(np.diff(E) <= 1e-12 * E[0]) and E[-1] < 0.9 * E[0]
    # c_d = 0 is the plain scheme
    r0 = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, dt, 50, 0.0, lambda t: 0.0, u0=u0, c_d=0.0)
    r1 = stepper.run_sample(K, mn, np.zeros(m.n_dof), ~free, dt, 50, 0.0, lambda t: 0.0, u0=u0)
    assert np.array_equal(r0["u"], r1["u"])


def test_starter_first_step():
    m, kh, A, eh, h = tiny_case()
    K, mn, free, w2, phi = _modes(m, kh, A, eh, h)
    dt = 1e-6
    rng = np.random.default_rng(9)
    F = rng.normal(size=m.n_dof)
    for alpha in (0.0, 50.0):
        r = stepper.run_sample(K, mn, F, ~free, dt, 1, alpha, lambda t: 1.0)
        expect = np.where(free, 0.5 * dt * dt * F / np.repeat(mn, 3), 0.0)
        assert np.allclose(r["u"], expect, rtol=1e-14, atol=0)


def test_static_limit_under_damping():
    m, kh, A, eh, h = tiny_case()
    K, mn, free, w2, phi = _modes(m, kh, A, eh, h)
    alpha = 50.0
    dt = 0.9 * 2.0 / math.sqrt(w2[-1])
    rng = np.random.default_rng(10)
    F = rng.normal(size=m.n_dof) * 1e4
    t_end = 0.75
    n = int(math.ceil(t_end / dt))
    r = stepper.run_sample(K, mn, F, ~free, dt, n, alpha, lambda t: 1.0)
    us = _embed(free, spla.spsolve(K[free][:, free].tocsc(), F[free]))
    # slowest decay e^{-alpha t / 2}
    assert np.linalg.norm(r["u"] - us) <= 1e-7 * np.linalg.norm(us)
    assert math.exp(-0.5 * alpha * n * dt) < 1e-7


def test_load_factor_shapes():
    assert stepper.load_factor("step", 3.0) == 1.0
    assert stepper.load_factor("sine", 0.0, 0.05) == 0.0
    assert abs(stepper.load_factor("sine", 0.025, 0.05) - math.sqrt(0.5)) < 1e-15
    assert stepper.load_factor("sine", 0.06, 0.05) == 1.0
    assert abs(stepper.load_factor("sine_pulse", 0.25, 0.05, 1.0, 0.3) - 1.3) < 1e-15
