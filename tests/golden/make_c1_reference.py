"""Write tests/golden/c1_reference.npz: the oracle's C1 run to 100,000 steps.

Workload: straight clamped cylinder R = 1 cm, L = 10 cm, 40 x 20 nodes,
S = 8 lognormal Matern fields (dense Cholesky on centroids, seed 1), nu =
0.49, k = 5/6, rho = 1, alpha = 50 1/s, uniform pressure 1.33e5 dyn/cm^2
under a 0.05 s sine ramp, dt = 0.9 x the element-eigenvalue bound.

Only the oracle and the seeded input generators are called.  Run from the
repository root:  python tests/golden/make_c1_reference.py
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2101_09059_amd import inputs  # noqa: E402
from oracle import assembly, cfl, element, matern, stepper  # noqa: E402

N_STEPS = 100_000
CHECKPOINTS = tuple(range(10_000, N_STEPS + 1, 10_000))


def setup():
    c = inputs.CONFIGS["c1_tiny"]
    m = inputs.cylinder(c["R"], c["L"], c["n_theta"], c["n_z"])
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, c["nu"], c["shear_k"])
    eh, h = matern.lognormal_fields(m.xyz, m.tri, c["S"], c["seed"])
    dt = cfl.stable_dt(kh, A, eh, h, c["rho"], c["safety"])
    F = inputs.traction_load(m, c["p0"])
    return c, m, kh, A, eh, h, dt, F


def one(s):
    c, m, kh, A, eh, h, dt, F = setup()
    g = lambda t: stepper.load_factor(c["ramp"], t, c["T_ramp"])
    r = stepper.run_ensemble(m.tri, kh, A, eh, h, c["rho"], F, m.fixed, m.radial, dt, N_STEPS,
                             c["alpha"], g, checkpoints=CHECKPOINTS, samples=[s])
    return r


def main():
    c, m, kh, A, eh, h, dt, F = setup()
    with Pool(min(8, c["S"])) as pool:
        res = pool.map(one, range(c["S"]))
    cps = np.stack([np.concatenate([r["checkpoints"][k] for r in res], axis=1) for k in CHECKPOINTS])
    q = np.concatenate([r["q"] for r in res], axis=1)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_reference.npz")
    np.savez_compressed(out, dt=dt, steps=np.array(CHECKPOINTS), u=cps, q=q)
    print("wrote", out, "dt", dt)


if __name__ == "__main__":
    main()
