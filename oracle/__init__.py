"""Plain FP64 CPU oracle for the ensemble wall solver -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (the HIP library and its binding)
never calls it and shares no code with it.

What it computes, following the paper (arXiv 2101.09059, Li & Schiavazzi):
  * element.py  -- 3-dof shell element: local frame, strain matrix B,
                   constitutive matrix C, element stiffness (Sec. 2.2.1);
  * assembly.py -- per-sample global stiffness K_s = sum_e (E h)_{e,s} P_e^T
                   K^_e P_e as a scipy CSR matrix and the lumped mass
                   (Sec. 2.2.1, Sec. 2.3);
  * stepper.py  -- central-difference update with lumped mass and
                   mass-proportional damping, one sample at a time
                   (Sec. 2.3, eq. dynamicsCD); running peak radial
                   displacement and the discrete energy;
  * cfl.py      -- stable step from the largest element eigenvalue;
  * matern.py   -- Matern covariance and dense-Cholesky field samples on
                   element centroids (Sec. 2.1);
  * stats.py    -- per-node ensemble mean and variance;
  * mlp.py      -- the learned form's GELU network, forward / backward / Adam;
  * control_variate.py -- multifidelity control-variate mean / variance
                   and its fallback rule;
  * stress.py   -- wall stresses in the local cylindrical frame (Sec. 2.3)
                   and their ensemble mean / quantile bands;
  * geometry.py -- stiffness rebuilt on the moved geometry (geometry update
                   with selective refresh, Sec. 2.3);
  * spde.py     -- Matern fields from the SPDE / GMRF formulation (Sec. 2.1).

Every function is pinned by the CPU tests (closed forms, invariants,
textbook special cases); see each module header for its pins.
"""
