"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Tolerances: FP64 path 1e-10 relative L2 over the [n_dof x S] block (at the
final step and at 10 checkpoints); FP32 apply with FP64 or Kahan-compensated
FP32 state 1e-5.  Apply-only: FP64 1e-13, FP32 1e-5 per sample.
"""
import math

import numpy as np
import pytest

from oracle import stats, stepper, cfl
from paper_2101_09059_amd import ensfem, inputs
from tests._cases import c1_case, small_case, say, rel_l2, oracle_apply, per_sample_max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(cs, **kw):
    kw.setdefault("alpha", 50.0)
    return ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, **kw)


def test_cfl_dt_matches_oracle():
    cs = c1_case()
    say("case: C1 cfl")
    ens = _ctx(cs)
    assert abs(ens.cfl_dt(0.9) / cs.dt - 1.0) < 1e-12
    ens.close()


@pytest.mark.parametrize("nt,nz,S", [(40, 20, 8), (37, 23, 13), (16, 9, 1), (30, 12, 100), (24, 10, 64),
                                     (48, 30, 200)])
@pytest.mark.parametrize("prec", [ensfem.F64, ensfem.F32])
def test_apply_parity(nt, nz, S, prec):
    say(f"case: apply nt={nt} nz={nz} S={S} prec={prec}")
    cs = small_case(nt, nz, S, seed=nt * 7 + S)
    ens = _ctx(cs)
    info = ens.info()
    ld = info["S_pad"]
    rng = np.random.default_rng(S)
    U = rng.standard_normal((cs.mesh.n_dof, S))
    dt = torch.float64 if prec == ensfem.F64 else torch.float32
    Ud = torch.zeros((cs.mesh.n_dof, ld), dtype=dt, device="cuda")
    Ud[:, :S] = torch.from_numpy(U).to(dt)
    Rd = torch.full((cs.mesh.n_dof, ld), float("nan"), dtype=dt, device="cuda")
    ens.apply(Ud, Rd, prec)
    torch.cuda.synchronize()
    R = Rd[:, :S].double().cpu().numpy()
    Uo = Ud[:, :S].double().cpu().numpy()  # the exact input the kernel saw
    ref = oracle_apply(cs, Uo)
    tol = 1e-13 if prec == ensfem.F64 else 1e-5
    for s in range(S):
        assert np.linalg.norm(R[:, s] - ref[:, s]) <= tol * np.linalg.norm(ref[:, s]), s
    ens.close()


def _run_gpu(cs, n_total, chunk, **kw):
    ens = _ctx(cs, kind=ensfem.LOAD_RAMP_SINE, t_ramp=cs.cfg["T_ramp"], **kw)
    ens.init_state()
    cps = {}
    done = 0
    while done < n_total:
        ens.step(chunk, cs.dt)
        done += chunk
        cps[done] = ens.read_state()
    q = ens.read_qoi()
    mean, var = ens.moments()
    ens.close()
    return cps, q, mean, var


def test_c1_fp64_2000_steps_vs_oracle():
    cs = c1_case()
    c = cs.cfg
    say("case: C1 FP64 2000 steps")
    cps, q, mean, var = _run_gpu(cs, 2000, 200)
    ref = stepper.run_ensemble(cs.mesh.tri, cs.khat, cs.area, cs.eh, cs.h, c["rho"], cs.F, cs.mesh.fixed,
                               cs.mesh.radial, cs.dt, 2000, c["alpha"], cs.g,
                               checkpoints=tuple(range(200, 2001, 200)))
    for n, u in cps.items():
        assert rel_l2(u, ref["checkpoints"][n]) <= 1e-10, n
        assert per_sample_max_rel(u, ref["checkpoints"][n]) <= 1e-10, n
    assert rel_l2(q, ref["q"]) <= 1e-10
    assert per_sample_max_rel(q, ref["q"]) <= 1e-10
    m_ref, v_ref = stats.moments(ref["q"])
    assert rel_l2(mean, m_ref) <= 1e-10
    assert rel_l2(var, v_ref) <= 1e-9


@pytest.mark.parametrize("mode,tol", [("f64", 1e-10), ("f32_kahan", 1e-5), ("f32_apply_f64_state", 1e-5)])
def test_c1_100k_steps_vs_golden(mode, tol):
    g = np.load("tests/golden/c1_reference.npz")
    cs = c1_case()
    assert cs.dt == float(g["dt"])
    kw = dict(f64={}, f32_kahan=dict(apply_prec=ensfem.F32, state_prec=ensfem.STATE_F32_KAHAN),
              f32_apply_f64_state=dict(apply_prec=ensfem.F32))[mode]
    say(f"case: C1 100k steps {mode}")
    cps, q, _, _ = _run_gpu(cs, 100_000, 10_000, **kw)
    errs = [rel_l2(cps[int(n)], g["u"][i]) for i, n in enumerate(g["steps"])]
    worst = [per_sample_max_rel(cps[int(n)], g["u"][i]) for i, n in enumerate(g["steps"])]
    say(f"  {mode}: rel L2 per checkpoint {['%.2e' % e for e in errs]}")
    say(f"  {mode}: per-sample max per checkpoint {['%.2e' % e for e in worst]}")
    assert max(errs) <= tol
    assert max(worst) <= tol
    assert rel_l2(q, g["q"]) <= tol
    assert per_sample_max_rel(q, g["q"]) <= tol


def test_c1_plain_fp32_state_is_worse_than_kahan():
    g = np.load("tests/golden/c1_reference.npz")
    cs = c1_case()
    say("case: C1 100k steps plain FP32 state")
    cps, _, _, _ = _run_gpu(cs, 100_000, 50_000, apply_prec=ensfem.F32, state_prec=ensfem.STATE_F32)
    cpk, _, _, _ = _run_gpu(cs, 100_000, 50_000, apply_prec=ensfem.F32, state_prec=ensfem.STATE_F32_KAHAN)
    e_plain = rel_l2(cps[100_000], g["u"][-1])
    e_kahan = rel_l2(cpk[100_000], g["u"][-1])
    say(f"  plain FP32 state {e_plain:.3e}  Kahan {e_kahan:.3e}")
    # on this coarse mesh the FP32 apply's own error (a few 1e-7) is the
    # floor of both states; the compensation still has to show
    assert np.isfinite(e_plain) and e_kahan <= 0.75 * e_plain


def test_nonzero_initial_state_and_pulsatile_load():
    cs = small_case(20, 12, 6, seed=3)
    rng = np.random.default_rng(4)
    free = ~cs.mesh.fixed.reshape(-1).astype(bool)
    u0 = rng.standard_normal((cs.mesh.n_dof, 6)) * 1e-3 * free[:, None]
    v0 = rng.standard_normal((cs.mesh.n_dof, 6)) * 1e-1 * free[:, None]
    n = 3000
    g = lambda t: stepper.load_factor("sine_pulse", t, 0.01, 0.02, 0.3)
    ref = []
    from oracle import assembly
    for s in range(6):
        K = assembly.assemble_stiffness(cs.mesh.tri, cs.khat, cs.eh[:, s], cs.mesh.n_nodes)
        m = assembly.lumped_mass(cs.mesh.tri, cs.area, cs.h[:, s], 1.0, cs.mesh.n_nodes)
        ref.append(stepper.run_sample(K, m, cs.F.reshape(-1), ~free, cs.dt, n, 20.0, g,
                                      u0=u0[:, s], v0=v0[:, s])["u"])
    ref = np.stack(ref, axis=1)
    for mode, tol, kw in [("f64", 1e-10, {}),
                          ("kahan", 1e-5, dict(apply_prec=ensfem.F32, state_prec=ensfem.STATE_F32_KAHAN))]:
        say(f"case: nonzero start + pulsatile, {mode}")
        ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, alpha=20.0, kind=ensfem.LOAD_PULSATILE,
                                t_ramp=0.01, amp=0.3, period=0.02, **kw)
        ens.init_state(u0, v0)
        ens.step(n, cs.dt)
        u = ens.read_state()
        ens.close()
        assert rel_l2(u, ref) <= tol, mode


def test_explicit_viscous_force_matches_oracle():
    """The explicit viscous force -c_d (u_n - u_{n-1}) / dt (and -c_d v_0 in
    the starter) against the oracle, from a moving start under a ramped load,
    for the FP64, FP32-apply / FP64-state and Kahan-FP32 paths."""
    cs = small_case(24, 14, 6, seed=8)
    rng = np.random.default_rng(9)
    free = ~cs.mesh.fixed.reshape(-1).astype(bool)
    u0 = rng.standard_normal((cs.mesh.n_dof, 6)) * 1e-3 * free[:, None]
    v0 = rng.standard_normal((cs.mesh.n_dof, 6)) * 1e-1 * free[:, None]
    from oracle import assembly
    m_min = min(assembly.lumped_mass(cs.mesh.tri, cs.area, cs.h[:, s], 1.0, cs.mesh.n_nodes).min()
                for s in range(6))
    c_d = 0.05 * m_min / cs.dt
    n = 2000
    g = lambda t: stepper.load_factor("sine", t, 0.01)
    ref = []
    for s in range(6):
        K = assembly.assemble_stiffness(cs.mesh.tri, cs.khat, cs.eh[:, s], cs.mesh.n_nodes)
        m = assembly.lumped_mass(cs.mesh.tri, cs.area, cs.h[:, s], 1.0, cs.mesh.n_nodes)
        ref.append(stepper.run_sample(K, m, cs.F.reshape(-1), ~free, cs.dt, n, 10.0, g,
                                      u0=u0[:, s], v0=v0[:, s], c_d=c_d)["u"])
    ref = np.stack(ref, axis=1)
    plain = []
    for s in range(6):
        K = assembly.assemble_stiffness(cs.mesh.tri, cs.khat, cs.eh[:, s], cs.mesh.n_nodes)
        m = assembly.lumped_mass(cs.mesh.tri, cs.area, cs.h[:, s], 1.0, cs.mesh.n_nodes)
        plain.append(stepper.run_sample(K, m, cs.F.reshape(-1), ~free, cs.dt, n, 10.0, g,
                                        u0=u0[:, s], v0=v0[:, s])["u"])
    assert rel_l2(np.stack(plain, axis=1), ref) > 1e-3  # the force matters at this c_d
    for mode, tol, kw in [("f64", 1e-10, {}),
                          ("f32 apply", 1e-5, dict(apply_prec=ensfem.F32)),
                          ("kahan", 1e-5, dict(apply_prec=ensfem.F32, state_prec=ensfem.STATE_F32_KAHAN))]:
        say(f"case: viscous force c_d={c_d:.3e}, {mode}")
        ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, alpha=10.0, kind=ensfem.LOAD_RAMP_SINE,
                                t_ramp=0.01, c_d=c_d, **kw)
        ens.init_state(u0, v0)
        ens.step(n, cs.dt)
        u = ens.read_state()
        ens.close()
        err = rel_l2(u, ref)
        say(f"  rel L2 {err:.2e}")
        assert err <= tol, mode


def test_mass_scaling_matches_oracle():
    """Mass scaling to 1.5x the unscaled stable step: the library's bound
    gives the target, and stepping at 0.99 of it matches the oracle run with
    the scaled lumped masses (FP64)."""
    S = 4
    cs = small_case(28, 12, S, seed=13)
    from oracle import assembly
    dt0 = cfl.stable_dt(cs.khat, cs.area, cs.eh, cs.h, 1.0, 1.0)
    dt_t = 1.5 * dt0
    f = cfl.mass_scale_factors(cs.khat, cs.area, cs.eh, cs.h, 1.0, dt_t)
    say(f"case: mass scaling to {dt_t:.3e} ({(f > 1).mean():.2%} of element-samples scaled)")
    ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, alpha=50.0, kind=ensfem.LOAD_RAMP_SINE, t_ramp=5e-3,
                            mass_dt=dt_t)
    assert abs(ens.cfl_dt(1.0) / dt_t - 1.0) < 1e-12
    dt = 0.99 * dt_t
    n = 1500
    ens.init_state()
    ens.step(n, dt)
    u = ens.read_state()
    ens.close()
    free = ~cs.mesh.fixed.reshape(-1).astype(bool)
    g = lambda t: stepper.load_factor("sine", t, 5e-3)
    ref = []
    for s in range(S):
        K = assembly.assemble_stiffness(cs.mesh.tri, cs.khat, cs.eh[:, s], cs.mesh.n_nodes)
        m = assembly.lumped_mass(cs.mesh.tri, cs.area, cs.h[:, s], 1.0, cs.mesh.n_nodes, f[:, s])
        ref.append(stepper.run_sample(K, m, cs.F.reshape(-1), ~free, dt, n, 50.0, g)["u"])
    ref = np.stack(ref, axis=1)
    assert np.all(np.isfinite(u))
    assert rel_l2(u, ref) <= 1e-10


def test_energy_conserved_and_matches_oracle():
    cs = small_case(18, 10, 4, seed=5)
    free = ~cs.mesh.fixed.reshape(-1).astype(bool)
    rng = np.random.default_rng(6)
    u0 = rng.standard_normal((cs.mesh.n_dof, 4)) * 1e-3 * free[:, None]
    F0 = np.zeros_like(cs.F)
    n = 1000
    say("case: energy conservation, undamped, unforced")
    ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, F0, alpha=0.0, energy_every=10)
    ens.init_state(u0)
    ens.step(n, cs.dt)
    ens.sync()  # the energy watchdog stays quiet on a stable run from a rough start
    steps, E = ens.read_energy()
    ens.close()
    assert len(steps) == n // 10 and steps[0] == 0 and steps[-1] == n - 10
    from oracle import assembly
    for s in range(4):
        K = assembly.assemble_stiffness(cs.mesh.tri, cs.khat, cs.eh[:, s], cs.mesh.n_nodes)
        m = assembly.lumped_mass(cs.mesh.tri, cs.area, cs.h[:, s], 1.0, cs.mesh.n_nodes)
        r = stepper.run_sample(K, m, np.zeros(cs.mesh.n_dof), ~free, cs.dt, n, 0.0, lambda t: 0.0,
                               u0=u0[:, s], energy_every=10)
        e_ref = np.array([e for _, e in r["energy"]])
        assert np.max(np.abs(E[:, s] - e_ref)) <= 1e-10 * abs(e_ref[0])
        assert np.max(np.abs(E[:, s] - E[0, s])) <= 1e-11 * abs(E[0, s])


@pytest.mark.parametrize("state", [ensfem.STATE_F64, ensfem.STATE_F32_KAHAN])
def test_energy_watchdog_flags_an_unstable_step(state):
    """Energy records every 10 steps on the C1 cylinder: at the stable step
    and at a step forced 5 % past the element bound (still below the
    assembled system's limit, about 1.2 times the bound here) ens_sync is
    quiet; forced 1.6 times past the bound the highest modes grow, and
    ens_sync reports ENS_EUNSTABLE from the watchdog well before the state
    overflows; a new initial state clears it."""
    cs = c1_case()
    kw = dict(kind=ensfem.LOAD_RAMP_SINE, t_ramp=cs.cfg["T_ramp"], energy_every=10, state_prec=state,
              apply_prec=ensfem.F64 if state == ensfem.STATE_F64 else ensfem.F32)
    bound = cs.dt / cs.cfg["safety"]
    for factor, unstable in ((cs.cfg["safety"], False), (1.05, False), (1.6, True)):
        say(f"case: watchdog state={state} dt = {factor} x bound")
        ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, **kw)
        ens.init_state()
        ens.step(50, factor * bound, force=True)
        if unstable:
            with pytest.raises(ensfem.EnsfemError) as ei:
                ens.sync()
            assert ei.value.code == ensfem.ENS_EUNSTABLE
            assert np.all(np.isfinite(ens.read_state()))  # caught before any overflow
            ens.init_state()
            ens.step(0, cs.dt)
            ens.sync()
        else:
            ens.sync()
        ens.close()


@pytest.mark.parametrize("state", [ensfem.STATE_F64, ensfem.STATE_F32_KAHAN])
def test_checkpoint_resume_is_bitwise(state):
    cs = c1_case()
    kw = dict(kind=ensfem.LOAD_RAMP_SINE, t_ramp=0.05, state_prec=state,
              apply_prec=ensfem.F64 if state == ensfem.STATE_F64 else ensfem.F32)
    say(f"case: checkpoint state={state}")
    a = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, **kw)
    a.init_state()
    a.step(1000, cs.dt)
    full = a.read_state()
    qa = a.read_qoi()
    a.close()
    b = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, **kw)
    b.init_state()
    b.step(500, cs.dt)
    blob = b.save()
    b.close()
    c = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, **kw)
    c.load(blob)
    c.step(500, cs.dt)
    assert np.array_equal(c.read_state(), full)
    assert np.array_equal(c.read_qoi(), qa)
    c.close()


def test_error_paths():
    cs = small_case(10, 6, 2)
    m = cs.mesh
    say("case: error paths")
    ens = ensfem.Ensemble(0)
    bad_tri = m.tri.copy()
    bad_tri[3, 1] = m.n_nodes + 5
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.set_mesh(m.xyz, bad_tri, m.fixed, m.radial)
    assert ei.value.code == ensfem.ENS_EINVAL
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.set_mesh(m.xyz, m.tri, m.fixed, 2.0 * m.radial)
    assert ei.value.code == ensfem.ENS_EINVAL
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.set_ensemble(cs.eh, cs.h)
    assert ei.value.code == ensfem.ENS_ESTATE
    ens.set_mesh(m.xyz, m.tri, m.fixed, m.radial)
    eh = cs.eh.copy()
    eh[2, 1] = np.nan
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.set_ensemble(eh, cs.h)
    assert ei.value.code == ensfem.ENS_EINVAL
    ens.set_material(0.49, 5 / 6, 1.0, 0.0)
    ens.set_ensemble(cs.eh, cs.h)
    ens.set_load(cs.F)
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.step(1, cs.dt)
    assert ei.value.code == ensfem.ENS_EWORKSPACE
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.bind_workspace(small)
    assert ei.value.code == ensfem.ENS_EWORKSPACE
    ens.bind_workspace()
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.step(1, cs.dt)
    assert ei.value.code == ensfem.ENS_ESTATE
    ens.init_state()
    bound = ens.cfl_dt(1.0)
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.step(1, 1.01 * bound)
    assert ei.value.code == ensfem.ENS_EUNSTABLE
    ens.step(10, cs.dt)
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.step(1, 0.5 * cs.dt)
    assert ei.value.code == ensfem.ENS_EINVAL
    ens.sync()
    # forcing an unstable step size: the watchdog reports non-finite values
    ens.init_state()
    ens.step(3000, 3.0 * bound, force=True)
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.sync()
    assert ei.value.code == ensfem.ENS_ENONFINITE
    ens.close()


def test_c2_full_size_sampled_columns():
    """The bench workload (400 x 500 cylinder, S = 256) in the bench's launch
    configuration, FP64 and FP32 apply, 2,000 steps (about 2.7 periods of
    the wall's breathing mode, past the starter transient), three sample
    columns checked against the oracle, which runs them in three CPU worker
    processes while the GPU steps."""
    import multiprocessing as mp
    from tests._cases import c2_oracle_column
    c = inputs.CONFIGS["c2_cylinder"]
    n, cols = 2000, [0, 137, 255]
    say(f"case: C2 full size, {n} steps, oracle columns {cols} in worker processes")
    pool = mp.get_context("spawn").Pool(len(cols))
    pending = pool.map_async(c2_oracle_column, [(col, n) for col in cols])
    pool.close()
    m = inputs.cylinder(c["R"], c["L"], c["n_theta"], c["n_z"])
    eh, h = inputs.lognormal_fields(m, c["S"], c["seed"])
    F = inputs.traction_load(m, c["p0"])
    from oracle import element
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, c["nu"], c["shear_k"])
    dt = cfl.stable_dt(kh, A, eh, h, c["rho"], c["safety"])
    got = {}
    for apply_prec in (ensfem.F64, ensfem.F32):
        say(f"  GPU run apply_prec={apply_prec}")
        ens = ensfem.setup_case(m, eh, h, F, alpha=c["alpha"], apply_prec=apply_prec)
        assert abs(ens.cfl_dt(0.9) / dt - 1) < 1e-12
        ens.init_state()
        ens.step(n, dt)
        got[apply_prec] = (ens.read_state()[:, cols], ens.read_qoi()[:, cols])
        ens.close()
    say("  waiting for the oracle columns")
    res = pending.get(timeout=600)
    pool.join()
    ref_u = np.stack([r[0] for r in res], axis=1)
    ref_q = np.stack([r[1] for r in res], axis=1)
    for apply_prec, tol in ((ensfem.F64, 1e-10), (ensfem.F32, 1e-5)):
        u, q = got[apply_prec]
        eu, es, eq = rel_l2(u, ref_u), per_sample_max_rel(u, ref_u), rel_l2(q, ref_q)
        say(f"  apply_prec={apply_prec}: rel L2 u {eu:.2e} (per-sample max {es:.2e}), q {eq:.2e}")
        assert eu <= tol and es <= tol and eq <= tol


@pytest.mark.parametrize("sb", [64, 128, 256])
@pytest.mark.parametrize("prec", [ensfem.F64, ensfem.F32])
def test_apply_parity_wide_sample_blocks(sb, prec):
    """2 and 4 consecutive samples per lane (vector loads), ragged S."""
    S = 200
    say(f"case: apply wide sb={sb} prec={prec} S={S}")
    cs = small_case(33, 17, S, seed=sb)
    ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, sample_block=sb)
    ld = ens.info()["S_pad"]
    assert ld % sb == 0 and ens.info()["sample_block"] == sb
    rng = np.random.default_rng(sb)
    dt = torch.float64 if prec == ensfem.F64 else torch.float32
    Ud = torch.zeros((cs.mesh.n_dof, ld), dtype=dt, device="cuda")
    Ud[:, :S] = torch.from_numpy(rng.standard_normal((cs.mesh.n_dof, S))).to(dt)
    Rd = torch.full((cs.mesh.n_dof, ld), float("nan"), dtype=dt, device="cuda")
    ens.apply(Ud, Rd, prec)
    torch.cuda.synchronize()
    R = Rd[:, :S].double().cpu().numpy()
    ref = oracle_apply(cs, Ud[:, :S].double().cpu().numpy())
    tol = 1e-13 if prec == ensfem.F64 else 1e-5
    err = np.linalg.norm(R - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= tol
    ens.close()


@pytest.mark.parametrize("state,apply_prec", [(ensfem.STATE_F64, ensfem.F64), (ensfem.STATE_F32_KAHAN, ensfem.F32),
                                              (ensfem.STATE_F64, ensfem.F32)])
def test_step_bitwise_independent_of_sample_block(state, apply_prec):
    """Every (node, sample) does the same arithmetic in the same order
    whatever the lane mapping and workgroup size (the FP32 apply with the
    FP64 state runs 8-node workgroups at 128 and 256 samples per block, 4
    at 64 and at energy records), so the results must be bitwise equal."""
    cs = small_case(26, 14, 256, seed=11)
    kw = dict(state_prec=state, apply_prec=apply_prec, energy_every=7)
    outs = []
    for sb in (64, 128, 256):
        say(f"case: bitwise sb={sb} state={state} apply={apply_prec}")
        ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, sample_block=sb, **kw)
        ens.init_state()
        ens.step(300, cs.dt)
        outs.append((ens.read_state(), ens.read_qoi(), ens.read_energy()[1]))
        ens.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def _shared_case(nt, nz, S, seed):
    cs = small_case(nt, nz, S, seed=seed)
    cs.eh = np.repeat(cs.eh[:, :1], S, axis=1).copy()
    from oracle import cfl as _cfl
    cs.dt = _cfl.stable_dt(cs.khat, cs.area, cs.eh, cs.h, 1.0, 0.9)
    return cs


@pytest.mark.parametrize("prec", [ensfem.F64, ensfem.F32])
@pytest.mark.parametrize("S", [5, 128, 200])
def test_shared_stiffness_block_product(prec, S):
    """Shared (E h): K assembled once as 3x3 block rows, applied to the
    ensemble block; equals the oracle's K U and the element-by-element path."""
    say(f"case: shared-stiffness product S={S} prec={prec}")
    cs = _shared_case(29, 15, S, seed=S)
    ens = _ctx(cs)
    assert ens.info()["shared_stiffness"] == 1 and ens.info()["variant"] == ensfem.VARIANT_CSR_SHARED
    ld = ens.info()["S_pad"]
    dt = torch.float64 if prec == ensfem.F64 else torch.float32
    rng = np.random.default_rng(S + 1)
    Ud = torch.zeros((cs.mesh.n_dof, ld), dtype=dt, device="cuda")
    Ud[:, :S] = torch.from_numpy(rng.standard_normal((cs.mesh.n_dof, S))).to(dt)
    Rd = torch.empty_like(Ud)
    ens.apply(Ud, Rd, prec)
    eg = _ctx(cs, variant=ensfem.VARIANT_NODE_GATHER)
    Rg = torch.empty_like(Ud)
    eg.apply(Ud, Rg, prec)
    torch.cuda.synchronize()
    R = Rd[:, :S].double().cpu().numpy()
    ref = oracle_apply(cs, Ud[:, :S].double().cpu().numpy())
    tol = 1e-13 if prec == ensfem.F64 else 1e-5
    err = np.linalg.norm(R - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= tol
    Rgn = Rg[:, :S].double().cpu().numpy()
    assert (np.linalg.norm(R - Rgn, axis=0) / np.linalg.norm(Rgn, axis=0)).max() <= tol
    ens.close()
    eg.close()


@pytest.mark.parametrize("mode,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_shared_stiffness_time_stepping(mode, tol):
    cs = _shared_case(24, 14, 16, seed=9)
    kw = {} if mode == "f64" else dict(apply_prec=ensfem.F32)
    say(f"case: shared-stiffness stepping {mode}")
    ens = _ctx(cs, kind=ensfem.LOAD_RAMP_SINE, t_ramp=0.01, **kw)
    assert ens.info()["variant"] == ensfem.VARIANT_CSR_SHARED
    ens.init_state()
    n = 2000
    ens.step(n, cs.dt)
    u, q = ens.read_state(), ens.read_qoi()
    ens.close()
    g = lambda t: stepper.load_factor("sine", t, 0.01)
    ref = stepper.run_ensemble(cs.mesh.tri, cs.khat, cs.area, cs.eh, cs.h, 1.0, cs.F, cs.mesh.fixed,
                               cs.mesh.radial, cs.dt, n, 50.0, g)
    assert rel_l2(u, ref["u"]) <= tol
    assert rel_l2(q, ref["q"]) <= tol


def test_shared_variant_rejected_for_sample_dependent_stiffness():
    cs = small_case(12, 6, 4, seed=2)
    ens = ensfem.Ensemble(0)
    ens.set_mesh(cs.mesh.xyz, cs.mesh.tri, cs.mesh.fixed, cs.mesh.radial)
    ens.set_material(0.49, 5 / 6, 1.0, 50.0)
    ens.set_ensemble(cs.eh, cs.h)
    ens.set_load(cs.F)
    ens.configure(variant=ensfem.VARIANT_CSR_SHARED)
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.bind_workspace()
    assert ei.value.code == ensfem.ENS_EUNSUPPORTED
    ens.close()


def test_caller_numbering_invariance():
    """The library reorders nodes and elements internally; a caller that
    numbers the same mesh differently gets the same results in its own
    numbering (state, peak, moments, stand-alone apply), up to the rounding
    of a different summation order."""
    say("case: caller numbering invariance (33x17, S=24)")
    cs = small_case(33, 17, 24, seed=5)
    m = cs.mesh
    rng = np.random.default_rng(11)
    pn = rng.permutation(m.n_nodes)            # new caller index -> old node
    pe = rng.permutation(m.n_el)
    inv = np.empty_like(pn)
    inv[pn] = np.arange(m.n_nodes)
    m2 = inputs.Mesh(xyz=m.xyz[pn], tri=inv[m.tri[pe]].astype(np.int32), fixed=m.fixed[pn],
                     radial=m.radial[pn], axial=m.axial[pn], length=m.length, n_theta=m.n_theta,
                     n_z=m.n_z, name="permuted")
    u0 = 1e-4 * rng.standard_normal((m.n_dof, 24))
    u0.reshape(m.n_nodes, 3, 24)[m.fixed.astype(bool)] = 0.0
    u0_2 = u0.reshape(m.n_nodes, 3, 24)[pn].reshape(m.n_dof, 24)
    a = ensfem.setup_case(m, cs.eh, cs.h, cs.F, alpha=50.0, kind=ensfem.LOAD_RAMP_SINE, t_ramp=1e-3)
    b = ensfem.setup_case(m2, cs.eh[pe], cs.h[pe], cs.F[pn], alpha=50.0, kind=ensfem.LOAD_RAMP_SINE, t_ramp=1e-3)
    for e, u in ((a, u0), (b, u0_2)):
        e.init_state(u)
        e.step(300, cs.dt)
        e.sync()
    ua = a.read_state().reshape(m.n_nodes, 3, 24)[pn].reshape(m.n_dof, 24)
    assert rel_l2(b.read_state(), ua) < 1e-12
    assert rel_l2(b.read_qoi(), a.read_qoi()[pn]) < 1e-12
    (ma, va), (mb, vb) = a.moments(), b.moments()
    assert rel_l2(mb, ma[pn]) < 1e-12 and rel_l2(vb, va[pn]) < 1e-10
    ld = a.info()["S_pad"]
    U = torch.randn(m.n_dof, ld, dtype=torch.float64, device="cuda")
    U2 = U.view(m.n_nodes, 3, ld)[torch.as_tensor(pn, device="cuda")].reshape(m.n_dof, ld).contiguous()
    Ra, Rb = torch.empty_like(U), torch.empty_like(U)
    a.apply(U, Ra, ensfem.F64)
    b.apply(U2, Rb, ensfem.F64)
    torch.cuda.synchronize()
    Ra2 = Ra.view(m.n_nodes, 3, ld)[torch.as_tensor(pn, device="cuda")].reshape(m.n_dof, ld)
    assert float((Rb - Ra2).norm() / Ra2.norm()) < 1e-13
    with pytest.raises(ValueError):
        a.apply(U[:, :8].contiguous(), Ra, ensfem.F64)
    a.close()
    b.close()


def test_precision_ladder_on_a_fine_mesh():
    """Precision modes against the FP64 path on a fine mesh (28,800 nodes,
    element size ~0.026 cm on a 1 cm radius), 4,000 steps of a ramped load:
    the FP32 apply with an FP64 state stays within 1e-7; both FP32 states
    within 1e-5, and the compensated pair at most half the plain FP32
    state's error (the update is formed in FP64 for both, so the difference
    is the compensation of u's rounding)."""
    say("case: fine cylinder 240x120, S=8, 4000 steps, precision modes")
    cs = small_case(240, 120, 8, seed=21, R=1.0, L=2.0)
    out = {}
    for name, ap, st in (("ref", ensfem.F64, ensfem.STATE_F64), ("f64", ensfem.F32, ensfem.STATE_F64),
                         ("kahan", ensfem.F32, ensfem.STATE_F32_KAHAN), ("f32", ensfem.F32, ensfem.STATE_F32)):
        e = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, alpha=50.0, kind=ensfem.LOAD_RAMP_SINE, t_ramp=2e-3,
                              apply_prec=ap, state_prec=st)
        e.init_state()
        e.step(4000, cs.dt)
        e.sync()
        out[name] = e.read_state()
        e.close()
    err = {k: rel_l2(out[k], out["ref"]) for k in ("f64", "kahan", "f32")}
    say(f"  against FP64: " + ", ".join(f"{k} {v:.2e}" for k, v in err.items()))
    assert err["f64"] <= 1e-7
    assert err["kahan"] <= 1e-5 and err["f32"] <= 1e-5
    assert err["kahan"] <= 0.5 * err["f32"]


def test_degenerate_sizes():
    """One free triangle with one sample (a rigid drift under the load plus
    its membrane modes), zero steps leaving the state alone, and a single
    sample on a cylinder: FP64 against the oracle."""
    from oracle import assembly, element
    xyz = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    nrm = np.cross(xyz[1] - xyz[0], xyz[2] - xyz[0])
    nrm /= np.linalg.norm(nrm)
    m = inputs.Mesh(xyz=xyz, tri=tri, fixed=np.zeros((3, 3), dtype=np.uint8), radial=np.tile(nrm, (3, 1)),
                    axial=np.zeros(3), length=1.0, n_theta=3, n_z=1, name="one_triangle")
    kh, A, _ = element.reference_stiffness(xyz, tri, 0.49, 5.0 / 6.0)
    eh, h = np.array([[7e5]]), np.array([[0.1]])
    F = np.array([[1.0, 0.0, 2.0], [0.0, -1.0, 0.5], [0.3, 0.2, -1.0]]) * 1e3
    dt = cfl.stable_dt(kh, A, eh, h, 1.0, 0.5)
    say("case: one free triangle, S=1")
    ens = ensfem.setup_case(m, eh, h, F, alpha=10.0)
    ens.init_state()
    u0 = ens.read_state()
    ens.step(0, dt)
    assert np.array_equal(ens.read_state(), u0)
    ens.step(300, dt)
    u = ens.read_state()
    q = ens.read_qoi()
    ens.close()
    K = assembly.assemble_stiffness(tri, kh, eh[:, 0], 3)
    mass = assembly.lumped_mass(tri, A, h[:, 0], 1.0, 3)
    r = stepper.run_sample(K, mass, F.reshape(-1), np.zeros(9, bool), dt, 300, 10.0, lambda t: 1.0,
                           radial=m.radial)
    assert rel_l2(u[:, 0], r["u"]) <= 1e-10
    assert rel_l2(q[:, 0], r["q"]) <= 1e-10
    # one sample on a cylinder (padded to a block of 8)
    cs = small_case(18, 9, 1, seed=31)
    say("case: cylinder 18x9, S=1")
    ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, alpha=50.0, kind=ensfem.LOAD_RAMP_SINE, t_ramp=5e-3)
    ens.init_state()
    ens.step(500, cs.dt)
    u = ens.read_state()
    ens.close()
    g = lambda t: stepper.load_factor("sine", t, 5e-3)
    ref = stepper.run_ensemble(cs.mesh.tri, cs.khat, cs.area, cs.eh, cs.h, 1.0, cs.F, cs.mesh.fixed,
                               cs.mesh.radial, cs.dt, 500, 50.0, g)["u"]
    assert rel_l2(u, ref) <= 1e-10


@pytest.mark.parametrize("sb", [64, 128, 256])
def test_peak_tracking_through_many_turns(sb):
    """Undamped oscillation from a sudden load: the radial displacement
    turns many times and later tops stay below the first.  The peak is read
    back mid-run (while rises are open) and at the end, against the oracle's
    running maximum, at one, two and four samples per lane."""
    S = 70 if sb == 64 else 200
    cs = small_case(16, 8, S, seed=17)
    say(f"case: peak tracking, 16x8 S={S} block {sb}")
    ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, alpha=0.0, sample_block=sb)
    ens.init_state()
    ens.step(337, cs.dt)
    q_mid = ens.read_qoi()
    ens.step(663, cs.dt)
    q_end = ens.read_qoi()
    ens.close()
    g = lambda t: 1.0
    cols = [0, S // 2, S - 1]
    r_mid = stepper.run_ensemble(cs.mesh.tri, cs.khat, cs.area, cs.eh, cs.h, 1.0, cs.F, cs.mesh.fixed,
                                 cs.mesh.radial, cs.dt, 337, 0.0, g, samples=cols)
    r_end = stepper.run_ensemble(cs.mesh.tri, cs.khat, cs.area, cs.eh, cs.h, 1.0, cs.F, cs.mesh.fixed,
                                 cs.mesh.radial, cs.dt, 1000, 0.0, g, samples=cols)
    assert rel_l2(q_mid[:, cols], r_mid["q"]) <= 1e-10
    assert rel_l2(q_end[:, cols], r_end["q"]) <= 1e-10


@pytest.mark.parametrize("mode,tol", [("f64", 1e-10), ("f32_apply_f64_state", 1e-5), ("f32_kahan", 1e-5)])
def test_curved_tapered_tube_pulsatile_shear_vs_oracle(mode, tol):
    """The precision form's own workload at small size: the curved tapered
    tube (centreline arc of radius 8 cm, 20 cm long, radius 1.2 -> 0.6 cm) on
    a 24 x 96 node lattice, S = 16, the sine-ramped pulsatile pressure with
    the axial taper and the seeded 1 % wall shear (the workload's own load
    parameters), 2,000 steps, every sample column against the oracle."""
    c = inputs.CONFIGS["c3_curved"]
    m = inputs.curved_tube(24, 96)
    S = 16
    eh, h = inputs.lognormal_fields(m, S, c["seed"], radius=0.9)
    F = inputs.traction_load(m, c["p0"], axial_taper=c["axial_taper"], shear_frac=c["shear_frac"], seed=c["seed"])
    from oracle import element
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, c["nu"], c["shear_k"])
    dt = cfl.stable_dt(kh, A, eh, h, c["rho"], c["safety"])
    n = 2000
    kw = dict(f64={}, f32_apply_f64_state=dict(apply_prec=ensfem.F32),
              f32_kahan=dict(apply_prec=ensfem.F32, state_prec=ensfem.STATE_F32_KAHAN))[mode]
    say(f"case: curved tapered tube 24x96, S={S}, C3 load, {n} steps, {mode}")
    ens = ensfem.setup_case(m, eh, h, F, nu=c["nu"], shear_k=c["shear_k"], rho=c["rho"], alpha=c["alpha"],
                            kind=ensfem.LOAD_PULSATILE, t_ramp=c["T_ramp"], amp=c["pulse_amp"],
                            period=c["period"], **kw)
    assert abs(ens.cfl_dt(c["safety"]) / dt - 1) < 1e-12
    ens.init_state()
    ens.step(n, dt)
    u, q = ens.read_state(), ens.read_qoi()
    ens.close()
    g = lambda t: stepper.load_factor(c["ramp"], t, c["T_ramp"], c["period"], c["pulse_amp"])
    ref = stepper.run_ensemble(m.tri, kh, A, eh, h, c["rho"], F, m.fixed, m.radial, dt, n, c["alpha"], g)
    eu, es, eq = rel_l2(u, ref["u"]), per_sample_max_rel(u, ref["u"]), rel_l2(q, ref["q"])
    say(f"  rel L2 u {eu:.2e} (per-sample max {es:.2e}), q {eq:.2e}")
    assert eu <= tol and es <= tol and eq <= tol
