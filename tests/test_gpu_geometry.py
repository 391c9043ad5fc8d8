"""GPU geometry update with selective stiffness refresh (Sec. 2.3) against
the FP64 oracle, through the C ABI: each sample's element matrices on its
own moved geometry, rebuilt every few steps.  Tolerances as for the plain
step: 1e-10 relative L2 (FP64), 1e-5 (FP32 apply, FP64 state)."""
import numpy as np
import pytest

from oracle import stepper
from paper_2101_09059_amd import ensfem
from tests._cases import small_case, say, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NU, KS = 0.49, 5.0 / 6.0
LOADF = 0.2    # pressure scale: peak displacement ~5 % of the radius


def _oracle(cs, F, n, every, cols):
    g = lambda t: stepper.load_factor("sine", t, 20 * cs.dt)
    r = stepper.run_ensemble(cs.mesh.tri, cs.khat, cs.area, cs.eh, cs.h, 1.0, F, cs.mesh.fixed, cs.mesh.radial,
                             cs.dt, n, 50.0, g, samples=cols,
                             geometry=(cs.mesh.xyz, NU, KS, every) if every else None)
    return r["u"], r["q"]


# S = 6: 8 lanes per node; S = 70: a wave per node with one sample per lane
# (block 64) and two (the default block 128), ragged padded tail; S = 256
# with block 256: four samples per lane; a few sample columns checked
@pytest.mark.parametrize("nt,nz,S,cols,sb", [(20, 10, 6, None, 0), (16, 8, 70, [0, 33, 69], 64),
                                             (16, 8, 70, [0, 33, 69], 0), (16, 8, 256, [7, 200], 256)])
@pytest.mark.parametrize("every", [1, 7])
def test_geometry_refresh_matches_oracle(nt, nz, S, cols, sb, every):
    cs = small_case(nt, nz, S, seed=21)
    F = LOADF * cs.F
    n = 120 if every == 1 else 300
    ref_u, ref_q = _oracle(cs, F, n, every, cols)
    plain_u, _ = _oracle(cs, F, n, 0, cols)
    moved = rel_l2(plain_u, ref_u)
    say(f"case: geometry refresh every {every}, {nt}x{nz} S={S} block {sb}: refresh changes u by {moved:.2e}")
    assert moved > 1e-3   # the refresh matters at this load
    sel = slice(None) if cols is None else cols
    for mode, tol, kw in [("f64", 1e-10, {}), ("f32 apply", 1e-5, dict(apply_prec=ensfem.F32))]:
        ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, F, alpha=50.0, kind=ensfem.LOAD_RAMP_SINE,
                                t_ramp=20 * cs.dt, geom_every=every, sample_block=sb, **kw)
        ens.init_state()
        ens.step(n, cs.dt)
        ens.sync()
        u = ens.read_state()[:, sel]
        q = ens.read_qoi()[:, sel]
        ens.close()
        eu, eq = rel_l2(u, ref_u), rel_l2(q, ref_q)
        say(f"  {mode}: rel L2 u {eu:.2e}, peak radial {eq:.2e}")
        assert eu <= tol and eq <= tol, mode


def test_geometry_refresh_error_paths():
    cs = small_case(12, 6, 8, seed=2)
    say("case: geometry refresh error paths")
    ens = ensfem.Ensemble()
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.set_geometry_refresh(-1)
    assert ei.value.code == ensfem.ENS_EINVAL
    ens.close()
    for kw in (dict(apply_prec=ensfem.F32, state_prec=ensfem.STATE_F32_KAHAN), dict(energy_every=10)):
        ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, geom_every=5, **kw)
        ens.init_state()
        with pytest.raises(ensfem.EnsfemError) as ei:
            ens.step(3, cs.dt)
        assert ei.value.code == ensfem.ENS_EUNSUPPORTED
        ens.close()
    ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, geom_every=5)
    ens.init_state()
    ens.step(12, cs.dt)
    with pytest.raises(ensfem.EnsfemError) as ei:
        ens.save()
    assert ei.value.code == ensfem.ENS_EUNSUPPORTED
    with pytest.raises(ensfem.EnsfemError):
        ensfem.Batch([ens])
    # switching the refresh off again gives the plain step (re-bind needed)
    ens.set_geometry_refresh(0)
    ens.bind_workspace()
    ens.init_state()
    ens.step(12, cs.dt)
    ens.sync()
    ens.close()
