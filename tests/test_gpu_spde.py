"""GPU SPDE / GMRF Matern sampler (block conjugate gradients) against the
oracle's direct solve, through the C ABI."""
import math

import numpy as np
import pytest

from oracle import spde as ospde
from paper_2101_09059_amd import ensfem, inputs
from tests._cases import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


# S = 37, 64, 1 run one sample per lane, S = 100 two, S = 256 four; the
# 65 x 71 tube gives every wave several rows and a ragged last pair
@pytest.mark.parametrize("nt,nz,S", [(40, 30, 37), (24, 60, 64), (17, 9, 1), (31, 13, 100), (65, 71, 256)])
def test_samples_match_direct_solve(nt, nz, S):
    m = inputs.cylinder(1.0, 6.0, nt, nz)
    kappa = math.sqrt(2.0)
    z = np.random.default_rng(nt * 100 + S).standard_normal((m.n_nodes, S))
    say(f"case: spde {nt}x{nz} S={S}")
    sp = ensfem.Spde(m.xyz, m.tri, S)
    x, it, res = sp.sample(z, kappa, tol=1e-12, max_iter=5000)
    sp.close()
    ref = ospde.sample(m.xyz, m.tri, z, kappa)
    err = np.linalg.norm(x - ref, axis=0) / np.linalg.norm(ref, axis=0)
    say(f"  {it} iterations, relative residual {res:.1e}, max column error {err.max():.1e}")
    assert res <= 1e-12
    assert err.max() <= 1e-9


def test_sampler_is_reproducible():
    """Per-sample reductions run in a fixed order: a second call returns
    the same fields bit for bit."""
    m = inputs.cylinder(1.0, 6.0, 33, 41)
    z = np.random.default_rng(5).standard_normal((m.n_nodes, 256))
    say("case: spde reproducibility 33x41 S=256")
    sp = ensfem.Spde(m.xyz, m.tri, 256)
    x1, it1, _ = sp.sample(z, 1.3, tol=1e-10, max_iter=3000)
    x2, it2, _ = sp.sample(z, 1.3, tol=1e-10, max_iter=3000)
    sp.close()
    assert it1 == it2
    assert np.array_equal(x1, x2)


def test_fields_have_the_matern_variance():
    """Middle of a flat 16 x 16 square (rho = 2): the empirical variance of
    4,096 GPU samples at the central node against the discrete field's exact
    variance (within 4 standard errors) and the continuous Matern value."""
    n, side = 81, 16.0
    xs, ys = np.meshgrid(np.linspace(0, side, n), np.linspace(0, side, n))
    xyz = np.stack([xs.ravel(), ys.ravel(), np.zeros(n * n)], 1)
    tri = []
    for j in range(n - 1):
        for i in range(n - 1):
            a = j * n + i
            tri += [(a, a + 1, a + n + 1), (a, a + n + 1, a + n)]
    tri = np.array(tri, dtype=np.int32)
    kappa, S = math.sqrt(2.0), 4096
    z = np.random.default_rng(7).standard_normal((n * n, S))
    say("case: spde variance, 81x81 square, S=4096")
    sp = ensfem.Spde(xyz, tri, S)
    x, it, res = sp.sample(z, kappa, tol=1e-10, max_iter=5000)
    sp.close()
    c = (n // 2) * n + n // 2
    emp = float(np.var(x[c]))
    import scipy.sparse.linalg as spla
    K, C = ospde.operator(xyz, tri, kappa)
    w = spla.spsolve(K.tocsc(), np.eye(1, n * n, c).ravel())
    exact = float(np.sum(w * w * C))
    say(f"  {it} iterations; variance: empirical {emp:.4e}, discrete {exact:.4e}, "
        f"Matern {ospde.marginal_variance(kappa):.4e}")
    assert abs(emp / exact - 1.0) < 4 * math.sqrt(2.0 / (S - 1))
    assert abs(exact / ospde.marginal_variance(kappa) - 1.0) < 0.06  # 3.9 % discretisation error at this spacing


def test_rejects_bad_input():
    m = inputs.cylinder(1.0, 3.0, 10, 5)
    say("case: spde error paths")
    sp = ensfem.Spde(m.xyz, m.tri, 4)
    with pytest.raises(ValueError):
        sp.sample(np.zeros((m.n_nodes, 3)), 1.0)
    with pytest.raises(ensfem.EnsfemError):
        sp.sample(np.zeros((m.n_nodes, 4)), -1.0)
    x, it, res = sp.sample(np.zeros((m.n_nodes, 4)), 1.0)
    assert it == 0 and not x.any()
    sp.close()
    bad = m.tri.copy()
    bad[0, 0] = m.n_nodes + 5
    with pytest.raises(ensfem.EnsfemError):
        ensfem.Spde(m.xyz, bad, 4)
