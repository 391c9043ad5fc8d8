"""Batching form on the GPU: several meshes of uneven size and ensemble
width stepped by one launch per step (graph-captured loop); every mesh must
match its solo run bitwise, across graph replays, remainders, parity flips
and an autotuner pass, and sampled columns of every member must match the
FP64 oracle (1e-10 for the FP64 apply, 1e-5 for the FP32 apply)."""
import numpy as np
import pytest

from paper_2101_09059_amd import ensfem, inputs
from oracle import cfl, element, stepper
from tests._cases import say, rel_l2, per_sample_max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (n_theta, n_z, S): padded widths 64 .. 256 in steps of 64, two members
# padded to an odd multiple of 32 (32 and 160: a tail block of 32 samples)
# and one of 96 (one block of 96 samples on 48 lanes at 2 per lane)
SPECS = [(12, 8, 64), (30, 21, 128), (47, 40, 192), (17, 9, 256), (64, 33, 64), (20, 13, 32), (26, 17, 160),
         (22, 12, 96)]


T_RAMP = 0.003


def _member_inputs(i):
    nt, nz, S = SPECS[i]
    m = inputs.cylinder(0.5 + 0.1 * i, 3.0 + i, nt, nz)
    eh, h = inputs.lognormal_fields(m, S, seed=40 + i)
    F = inputs.traction_load(m, 1.33e5)
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, 0.49, 5.0 / 6.0)
    dt = cfl.stable_dt(kh, A, eh, h, 1.0, 0.9)
    return m, eh, h, F, kh, A, dt


def _members(apply_prec, state_prec):
    out = []
    for i, (nt, nz, S) in enumerate(SPECS):
        m, eh, h, F, kh, A, dt = _member_inputs(i)
        kw = dict(alpha=50.0, kind=ensfem.LOAD_RAMP_SINE, t_ramp=T_RAMP, apply_prec=apply_prec,
                  state_prec=state_prec, sample_block=64 if S % 64 == 0 else 32)
        a = ensfem.setup_case(m, eh, h, F, **kw)
        b = ensfem.setup_case(m, eh, h, F, **kw)
        out.append((a, b, dt))
    return out


def _start(pairs):
    for a, b, dt in pairs:
        for e in (a, b):
            e.init_state()
            e.step(0, dt)


@pytest.mark.parametrize("apply_prec,state_prec", [(ensfem.F32, ensfem.STATE_F64),
                                                   (ensfem.F64, ensfem.STATE_F64),
                                                   (ensfem.F32, ensfem.STATE_F32_KAHAN)])
def test_batch_matches_solo_bitwise(apply_prec, state_prec):
    say(f"case: batch vs solo apply={apply_prec} state={state_prec}")
    pairs = _members(apply_prec, state_prec)
    _start(pairs)
    batch = ensfem.Batch([b for _, b, _ in pairs])
    info = batch.info()
    assert info["n_meshes"] == len(SPECS) and info["graph_steps"] % 2 == 0
    for chunk in (100, 37, 64, 1, 200):
        say(f"  batch chunk {chunk}")
        batch.step(chunk)
        for a, b, dt in pairs:
            a.step(chunk, dt)
        for a, b, _ in pairs:
            assert np.array_equal(a.read_state(), b.read_state())
            assert np.array_equal(a.read_qoi(), b.read_qoi())
    # a solo step between batch calls flips one mesh's parity; on a member
    # padded to 160 it runs lane groups that keep the peak without rising
    # bits, so the rises the batch left open are folded in first
    for i in (1, 6):
        pairs[i][1].step(3, pairs[i][2])
        pairs[i][0].step(3, pairs[i][2])
    batch.step(130)
    for a, b, dt in pairs:
        a.step(130, dt)
        assert np.array_equal(a.read_state(), b.read_state())
    batch.close()
    for a, b, _ in pairs:
        a.close()
        b.close()


@pytest.mark.parametrize("spl,split,state_prec", [(1, 0, ensfem.STATE_F64), (1, 1, ensfem.STATE_F64),
                                                   (2, 0, ensfem.STATE_F64), (2, 1, ensfem.STATE_F64),
                                                   (2, 2, ensfem.STATE_F64), (1, 2, ensfem.STATE_F64),
                                                   (2, 2, ensfem.STATE_F32_KAHAN), (1, 1, ensfem.STATE_F32)])
def test_batch_tilings_match_solo_bitwise(spl, split, state_prec):
    """Every tiling (1 or 2 samples per lane; tail blocks in the same launch,
    their own, or their own on a second stream), switched between batch
    calls, gives the solo results bit for bit."""
    say(f"case: batch tiling spl={spl} split={split} state={state_prec}")
    pairs = _members(ensfem.F32, state_prec)
    _start(pairs)
    batch = ensfem.Batch([b for _, b, _ in pairs])
    for k, (s_, sp_) in enumerate([(spl, split), (3 - spl, (split + 1) % 3), (spl, split)]):
        batch.set_tiling(s_, sp_)
        n = (70, 33, 64)[k]
        say(f"  tiling {s_}/{sp_}: {batch.info()}, {n} steps")
        batch.step(n)
        for a, b, dt in pairs:
            a.step(n, dt)
        for a, b, _ in pairs:
            assert np.array_equal(a.read_state(), b.read_state())
            assert np.array_equal(a.read_qoi(), b.read_qoi())
    with pytest.raises(ensfem.EnsfemError):
        batch.set_tiling(3, 0)
    with pytest.raises(ensfem.EnsfemError):
        batch.set_tiling(2, 3)
    batch.close()
    for a, b, _ in pairs:
        a.close()
        b.close()


def test_batch_autotune_then_restart():
    say("case: batch autotune")
    pairs = _members(ensfem.F32, ensfem.STATE_F64)
    _start(pairs)
    batch = ensfem.Batch([b for _, b, _ in pairs])
    batch.autotune(4)
    info = batch.info()
    say(f"  tuned: {info}")
    assert info["tuned_ms_per_step"] > 0
    _start(pairs)
    batch.step(150)
    for a, b, dt in pairs:
        a.step(150, dt)
        assert np.array_equal(a.read_state(), b.read_state())
        assert np.array_equal(a.read_qoi(), b.read_qoi())
    batch.close()
    for a, b, _ in pairs:
        a.close()
        b.close()


def test_batch_rejects_incompatible_members():
    m = inputs.cylinder(1.0, 4.0, 12, 8)
    eh, h = inputs.lognormal_fields(m, 64, seed=3)
    F = inputs.traction_load(m, 1.0e5)
    a = ensfem.setup_case(m, eh, h, F, apply_prec=ensfem.F32)
    b = ensfem.setup_case(m, eh, h, F, apply_prec=ensfem.F64)
    with pytest.raises(ensfem.EnsfemError):
        ensfem.Batch([a, b])
    c = ensfem.setup_case(m, eh, h, F, apply_prec=ensfem.F32, energy_every=5)
    with pytest.raises(ensfem.EnsfemError):
        ensfem.Batch([a, c])
    for e in (a, b, c):
        e.close()


@pytest.mark.parametrize("apply_prec,tol", [(ensfem.F64, 1e-10), (ensfem.F32, 1e-5)])
def test_batch_members_match_oracle(apply_prec, tol):
    """After an autotuner pass, 301 batched steps (graph replays plus an odd
    remainder; both lane classes: widths 64 and 192 have a tail block of 64
    samples, 32 and 160 one of 32, 96 a block of 96 on 48 lanes): the
    first, a middle and the last sample column of every member against the
    oracle's per-sample run."""
    say(f"case: batch vs oracle apply={apply_prec}")
    pairs = _members(apply_prec, ensfem.STATE_F64)
    _start(pairs)
    batch = ensfem.Batch([b for _, b, _ in pairs])
    batch.autotune(2)
    say(f"  tuned: {batch.info()}")
    _start(pairs)
    n = 301
    batch.step(n)
    g = lambda t: stepper.load_factor("sine", t, T_RAMP)
    for i, (a, b, dt) in enumerate(pairs):
        m, eh, h, F, kh, A, dt_o = _member_inputs(i)
        assert dt_o == dt
        S = SPECS[i][2]
        cols = [0, S // 2 + 1, S - 1]
        u, q = b.read_state()[:, cols], b.read_qoi()[:, cols]
        ref = stepper.run_ensemble(m.tri, kh, A, eh, h, 1.0, F, m.fixed, m.radial, dt, n, 50.0, g, samples=cols)
        eu, es, eq = rel_l2(u, ref["u"]), per_sample_max_rel(u, ref["u"]), rel_l2(q, ref["q"])
        say(f"  member {i} ({m.n_nodes} nodes, S={S}): rel L2 u {eu:.2e} (per-sample max {es:.2e}), q {eq:.2e}")
        assert eu <= tol and es <= tol and eq <= tol
    batch.close()
    for a, b, _ in pairs:
        a.close()
        b.close()
