"""Learned form end to end on a small cylinder: KL inputs, solver-generated
training data, GPU training, control variate against a large plain
reference, the gain over the plain estimator, and the fallback."""
import numpy as np
import pytest

from paper_2101_09059_amd import inputs, learned
from tests._cases import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CFG = dict(p0=1.33e5, T_ramp=0.02, period=1.0, pulse_amp=0.3, window=0.03, nu=0.49, shear_k=5.0 / 6.0,
           rho=1.0, alpha=50.0, safety=0.9)
N_MODES = 8
N_HF, N_LF, N_REF = 16384, 262144, 65536


@pytest.fixture(scope="module")
def setup():
    mesh = inputs.cylinder(1.0, 10.0, 24, 14)
    prob = learned.Problem(mesh, CFG, N_MODES)
    say(f"case: learned form, {mesh.n_nodes} nodes, KL captured {prob.captured:.3f}")
    Xtr = learned.draw_xi(5, 1024, N_MODES)
    Qtr = np.concatenate([prob.solve(Xtr[i:i + 256]) for i in range(0, 1024, 256)], axis=1).T
    net = learned.Network(2 * N_MODES, 128, 3, mesh.n_nodes, seed=9, max_batch=256)
    rmse, hist = net.fit(Xtr, Qtr, epochs=150, batch=128, lr=2e-3, seed=10)
    say(f"  held-out rel RMSE {rmse:.4f}, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    # The variance is judged within max(1 %, 2 SE_ref) of a 65,536-sample
    # reference (SE_ref 0.6 %), so the control variate's own error must be
    # well below that: N = 16,384 paired samples (at 1,024 its variance
    # carries about 1.5 % of its own) and M = 262,144 network draws.
    Xh = learned.draw_xi(6, N_HF, N_MODES)
    qH = np.concatenate([prob.solve(Xh[i:i + 256]) for i in range(0, N_HF, 256)], axis=1)
    pm, pv = qH.mean(axis=1), qH.var(axis=1, ddof=1)
    Xl = learned.draw_xi(7, N_LF, N_MODES)
    Xr = learned.draw_xi(8, N_REF, N_MODES)
    qR = np.concatenate([prob.solve(Xr[i:i + 256]) for i in range(0, N_REF, 256)], axis=1)
    yield dict(mesh=mesh, prob=prob, net=net, rmse=rmse, Xh=Xh, qH=qH, pm=pm, pv=pv, Xl=Xl, qR=qR)
    net.close()


def test_control_variate_matches_reference_and_gains(setup):
    s = setup
    net, qH = s["net"], s["qH"]
    assert s["rmse"] < 0.05
    qL = net.predict(s["Xh"]).T
    sumL, sumsqL = net.moment_sums(s["Xl"])
    M, N = s["Xl"].shape[0], qH.shape[1]
    est = learned.estimate(qH, s["pm"], s["pv"], qL, sumL, sumsqL, M, s["rmse"])
    say(f"  median rho {est['rho_median']:.4f}, used CV {est['used_cv']}")
    assert est["used_cv"]
    qR = s["qR"]
    act = qR.var(axis=1) > 0
    ref_m, ref_v = qR.mean(axis=1), qR.var(axis=1, ddof=1)
    Nr = qR.shape[1]
    se_m = np.linalg.norm(np.sqrt(ref_v[act] / Nr)) / np.linalg.norm(ref_m[act])
    e_cv = np.linalg.norm(est["mean"][act] - ref_m[act]) / np.linalg.norm(ref_m[act])
    e_plain = np.linalg.norm(s["pm"][act] - ref_m[act]) / np.linalg.norm(ref_m[act])
    e_var = np.linalg.norm(est["var"][act] - ref_v[act]) / np.linalg.norm(ref_v[act])
    # the reference variance's own standard error from its fourth moments
    d = qR[act] - ref_m[act][:, None]
    m2, m4 = (d * d).mean(axis=1), (d ** 4).mean(axis=1)
    se_v = np.linalg.norm(np.sqrt(np.maximum(m4 - m2 * m2, 0.0) / Nr)) / np.linalg.norm(ref_v[act])
    say(f"  mean rel err CV {e_cv:.2e} plain(N={N}) {e_plain:.2e} ref SE {se_m:.2e}; "
        f"var rel err {e_var:.2e} ref SE {se_v:.2e}")
    assert e_cv < max(0.01, 3 * se_m)
    assert e_var < max(0.01, 2 * se_v)
    # gain: variance ratio of the CV mean to the plain N-sample mean
    ratio = 1.0 - est["rho"][act] ** 2 * M / (M + N)
    gain = 1.0 / np.median(ratio)
    say(f"  predicted variance reduction x{gain:.1f}; equivalent plain samples {N * gain:.0f}")
    assert gain > 4.0
    assert e_cv < e_plain


def test_corrupted_network_falls_back_to_plain_statistics(setup):
    s = setup
    bad = learned.Network(2 * N_MODES, 128, 3, s["mesh"].n_nodes, seed=123, max_batch=256)
    bad.mu, bad.sd = s["net"].mu, s["net"].sd
    qL = bad.predict(s["Xh"]).T
    sumL, sumsqL = bad.moment_sums(s["Xl"])
    est = learned.estimate(s["qH"], s["pm"], s["pv"], qL, sumL, sumsqL, s["Xl"].shape[0], 0.5)
    assert not est["used_cv"]
    assert np.array_equal(est["mean"], s["pm"]) and np.array_equal(est["var"], s["pv"])
    bad.close()
