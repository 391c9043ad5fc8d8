"""Explicit central-difference time stepping, one sample at a time -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Equation of motion M u'' + C u' + K u = f(t) (Sec. 2.3), lumped M, damping
C = alpha M (mass-proportional), linear K.  The central-difference update of
eq. dynamicsCD with both mass matrices lumped reads, per dof,

    (1 + a) u_{n+1} = dt^2 (f_n - K u_n) / m + 2 u_n - (1 - a) u_{n-1},
    a = alpha dt / 2,

with clamped dofs held at zero and f_n = g(t_n) F, t_n = n dt.  The
optional explicit viscous force of Sec. 2.3, f_v = -c_d du/dt at t_n, is
added to f_n with the backward difference du/dt ~ (u_n - u_{n-1}) / dt
(one coefficient c_d per dof, the update stays explicit).

Optional geometry refresh (Sec. 2.3, oracle/geometry.py): with every > 0 the
internal force is carried incrementally, R_n = R_m + K_m (u_n - u_m), and
before steps m = every, 2 every, ... the base moves to R_m = R_{m'} +
K_{m'} (u_m - u_{m'}) and the matrix is rebuilt on the moved geometry,
K_m = K_at(u_m).

Start (the paper does not state one): u_0, v_0 given (zero = at rest) and
u_{-1} = u_0 - dt v_0 + dt^2/2 (M^-1 (f_0 - K u_0 - c_d v_0) - alpha v_0), the
Taylor start; for a ramped load that starts at zero this is u_{-1} = u_0 = 0.

Outputs: u_N (and u_{N-1}), optional checkpoints, the running peak radial
displacement q_i = max_{0<=n<=N} e_r,i . u_i(t_n), and the discrete energy
E_{n+1/2} = 1/2 v^T M v + 1/2 u_{n+1}^T K u_n, v = (u_{n+1} - u_n)/dt, which
the undamped, unforced scheme conserves exactly.

Pins (tests/test_oracle_stepper.py): single-mode closed form u_n = phi cos(n
theta) with cos theta = 1 - (omega dt)^2 / 2 (and the damped characteristic
roots), energy conservation and energy balance, monotone energy decay under
damping, convergence to the static K^-1 f, the starter's u_1, and the exact
discrete energy balance of the viscous force.
"""
from __future__ import annotations

import math
from typing import Callable, Optional, Sequence

import numpy as np

from . import assembly
from .geometry import IncrementalForce


def load_factor(kind: str, t: float, T_ramp: float = 0.0, period: float = 1.0, pulse_amp: float = 0.0) -> float:
    """Scalar time factor g(t) of the load f(t) = g(t) F.

    step        g = 1
    sine        g = sin(pi t / (2 T_ramp)) for t < T_ramp, else 1 (sine ramp, Sec. 3.1.2)
    sine_pulse  sine ramp times (1 + pulse_amp sin(2 pi t / period))
    """
    if kind == "step":
        return 1.0
    ramp = math.sin(math.pi * t / (2.0 * T_ramp)) if t < T_ramp else 1.0
    if kind == "sine":
        return ramp
    if kind == "sine_pulse":
        return ramp * (1.0 + pulse_amp * math.sin(2.0 * math.pi * t / period))
    raise ValueError(kind)


def run_sample(K, m_node: np.ndarray, F: np.ndarray, fixed: np.ndarray, dt: float, n_steps: int,
               alpha: float, g: Callable[[float], float], radial: Optional[np.ndarray] = None,
               u0: Optional[np.ndarray] = None, v0: Optional[np.ndarray] = None,
               u_prev: Optional[np.ndarray] = None, checkpoints: Sequence[int] = (),
               energy_every: int = 0, c_d: float = 0.0,
               K_at: Optional[Callable[[np.ndarray], object]] = None, every: int = 0,
               R_base: Optional[np.ndarray] = None, u_base: Optional[np.ndarray] = None):
    """Step one sample.  K: scipy sparse [n_dof, n_dof]; m_node [n_nodes];
    F [n_dof]; fixed [n_dof] bool.  If u_prev is given it is u_{-1} and the
    starter is skipped.  The internal force is R_base + K (u - u_base)
    (zero by default); with every > 0, before steps n = every, 2 every, ...
    R_base += K (u_n - u_base), u_base = u_n, K = K_at(u_n).  Returns a dict with u (u_N), u_prev (u_{N-1}),
    q (peak radial, [n_nodes]), checkpoints {n: u_n}, energy [(n, E_{n+1/2})]."""
    n_dof = K.shape[0]
    minv = np.repeat(1.0 / m_node, 3)
    a = 0.5 * alpha * dt
    u = np.zeros(n_dof) if u0 is None else np.array(u0, dtype=np.float64)
    u[fixed] = 0.0
    if u_prev is None:
        v = np.zeros(n_dof) if v0 is None else np.array(v0, dtype=np.float64)
        acc = minv * (g(0.0) * F - K @ u - c_d * v) - alpha * v
        u_prev = u - dt * v + 0.5 * dt * dt * acc
        u_prev[fixed] = 0.0
    else:
        u_prev = np.array(u_prev, dtype=np.float64)
    q = None
    if radial is not None:
        q = np.sum(radial * u.reshape(-1, 3), axis=1)
    cps = {}
    if 0 in checkpoints:
        cps[0] = u.copy()
    energy = []
    m_dof = np.repeat(m_node, 3)
    offset = R_base is not None or u_base is not None or every
    force = IncrementalForce(K, K_at, R_base, u_base)
    for n in range(n_steps):
        if every and n > 0 and n % every == 0:
            force.refresh(u)
        R = force.force(u) if offset else K @ u
        f = g(n * dt) * F - c_d * (u - u_prev) / dt
        u_next = (dt * dt * minv * (f - R) + 2.0 * u - (1.0 - a) * u_prev) / (1.0 + a)
        u_next[fixed] = 0.0
        if energy_every and (n % energy_every == 0):
            v = (u_next - u) / dt
            energy.append((n, 0.5 * np.dot(m_dof * v, v) + 0.5 * np.dot(u_next, R)))
        if q is not None:
            q = np.maximum(q, np.sum(radial * u_next.reshape(-1, 3), axis=1))
        u_prev, u = u, u_next
        if (n + 1) in checkpoints:
            cps[n + 1] = u.copy()
    return dict(u=u, u_prev=u_prev, q=q, checkpoints=cps, energy=energy, R_base=force.R_base,
                u_base=force.u_base)


def run_ensemble(tri: np.ndarray, khat: np.ndarray, area: np.ndarray, eh: np.ndarray, h: np.ndarray,
                 rho: float, F: np.ndarray, fixed: np.ndarray, radial: np.ndarray, dt: float,
                 n_steps: int, alpha: float, g: Callable[[float], float],
                 checkpoints: Sequence[int] = (), energy_every: int = 0,
                 samples: Optional[Sequence[int]] = None, c_d: float = 0.0, geometry=None):
    """S independent solves, sample by sample (no ensemble batching).
    eh, h [n_el, S]; F [n_nodes, 3]; fixed [n_nodes, 3]; radial [n_nodes, 3].
    Returns u [n_dof, S'], q [n_nodes, S'], checkpoints {n: [n_dof, S']},
    energy [S'] lists, for the chosen sample columns.  geometry = (xyz, nu,
    shear_k, every) turns on the geometry refresh."""
    n_nodes = radial.shape[0]
    cols = list(range(eh.shape[1])) if samples is None else list(samples)
    Fd = F.reshape(-1)
    fx = fixed.reshape(-1).astype(bool)
    us, qs, en = [], [], []
    cps = {c: [] for c in checkpoints}
    for s in cols:
        K = assembly.assemble_stiffness(tri, khat, eh[:, s], n_nodes)
        m = assembly.lumped_mass(tri, area, h[:, s], rho, n_nodes)
        kw = {}
        if geometry is not None:
            from . import geometry as geo
            xyz, nu, shear_k, every = geometry
            kw = dict(every=every, K_at=lambda u, s=s: geo.deformed_stiffness(xyz, tri, u, eh[:, s], nu, shear_k))
        r = run_sample(K, m, Fd, fx, dt, n_steps, alpha, g, radial=radial,
                       checkpoints=checkpoints, energy_every=energy_every, c_d=c_d, **kw)
        us.append(r["u"])
        qs.append(r["q"])
        en.append(r["energy"])
        for c in checkpoints:
            cps[c].append(r["checkpoints"][c])
    return dict(u=np.stack(us, axis=1), q=np.stack(qs, axis=1),
                checkpoints={c: np.stack(v, axis=1) for c, v in cps.items()}, energy=en)
