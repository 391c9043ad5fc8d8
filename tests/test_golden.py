"""The stored C1 reference (tests/golden/c1_reference.npz) is what the
oracle computes now: its step size, and its first checkpoint (10,000 steps)
for two sample columns, recomputed here."""
import importlib.util
import os

import numpy as np

from oracle import stepper

HERE = os.path.dirname(os.path.abspath(__file__))


def _maker():
    spec = importlib.util.spec_from_file_location("make_c1_reference",
                                                  os.path.join(HERE, "golden", "make_c1_reference.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_golden_file_matches_the_oracle():
    ref = np.load(os.path.join(HERE, "golden", "c1_reference.npz"))
    mk = _maker()
    c, m, kh, A, eh, h, dt, F = mk.setup()
    assert float(ref["dt"]) == dt
    first = int(ref["steps"][0])
    g = lambda t: stepper.load_factor(c["ramp"], t, c["T_ramp"])
    for s in (0, c["S"] - 1):
        r = stepper.run_ensemble(m.tri, kh, A, eh, h, c["rho"], F, m.fixed, m.radial, dt, first,
                                 c["alpha"], g, samples=[s])
        u_ref = ref["u"][0][:, s]
        err = np.linalg.norm(r["u"][:, 0] - u_ref) / np.linalg.norm(u_ref)
        assert err < 1e-12, (s, err)
