"""The allocation-free entry point ens_moments_noalloc against ens_moments
(same kernel, same summation order: bitwise equal), on two calls in a row
whose second has the smaller input, and its size limit."""
import numpy as np
import pytest

from paper_2101_09059_amd import ensfem, inputs
from tests._cases import c1_case, small_case, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _stepped(cs, n_steps, **kw):
    ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, alpha=50.0, kind=ensfem.LOAD_RAMP_SINE,
                            t_ramp=0.01, **kw)
    ens.init_state()
    ens.step(n_steps, cs.dt)
    ens.sync()
    return ens


def test_noalloc_moments_equal_ens_moments_on_two_calls():
    big = c1_case()  # 800 nodes, S = 8
    small = small_case(16, 9, 5, seed=3)  # 144 nodes, S = 5
    assert small.mesh.n_nodes < big.mesh.n_nodes
    for name, cs, n in (("C1 800 nodes S=8", big, 300), ("16x9 cylinder S=5", small, 120)):
        say(f"case: noalloc moments, {name}, {n} steps")
        ens = _stepped(cs, n)
        mean_ref, var_ref = ens.moments()
        mean = np.full(cs.mesh.n_nodes, np.nan)
        var = np.full(cs.mesh.n_nodes, np.nan)
        ens.moments_noalloc(mean, var)
        assert np.array_equal(mean, mean_ref)
        assert np.array_equal(var, var_ref)
        # the same values as the peak QoI read back and reduced on the host
        q = ens.read_qoi()
        np.testing.assert_allclose(mean, q.mean(axis=1), rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(var, q.var(axis=1, ddof=1), rtol=1e-10, atol=1e-300)
        ens.close()


def test_noalloc_moments_state_and_size_errors():
    say("case: noalloc moments errors")
    cs = small_case(12, 6, 2, seed=1)
    ens = ensfem.setup_case(cs.mesh, cs.eh, cs.h, cs.F, alpha=50.0)
    with pytest.raises(ensfem.EnsfemError) as ei:  # no state yet
        ens.moments_noalloc()
    assert ei.value.code == ensfem.ENS_ESTATE
    ens.close()
    # a mesh above the scratch limit (1,048,576 nodes) is refused before any
    # device work
    m = inputs.cylinder(1.0, 10.0, 1100, 1000)
    assert m.n_nodes > 1048576
    ctx = ensfem.Ensemble()
    ctx.set_mesh(m.xyz, m.tri, m.fixed, m.radial)
    with pytest.raises(ensfem.EnsfemError) as ei:
        ctx.moments_noalloc(np.empty(m.n_nodes), np.empty(m.n_nodes))
    assert ei.value.code == ensfem.ENS_EINVAL
    assert "scratch limit" in str(ei.value)
    ctx.close()
