/*
 * ensfem -- explicit-in-time ensemble solver for the three-dof linear shell
 * wall model (Li & Schiavazzi, arXiv 2101.09059), MI355X (gfx950) HIP library.
 *
 * One context = one wall mesh stepped for S material realizations at once
 * (Sec. 2.3-2.4).  Per step:  R = K(E h)_s U  (element stiffness of Sec. 2.2.1
 * scaled per element and sample by (E h)_{e,s}), then the lumped-mass
 * central-difference update with mass-proportional damping (eq.
 * dynamicsCD) under the wall-traction load f_n = g(t_n) F (Sec. 2.2.3).
 *
 * Conventions
 *  - Every call returns int32: ENS_OK (0) or a negative ENS_E* code.  The
 *    message of the last failure is ens_last_error(ctx) (valid until the
 *    next call on that context).  No C++ exception crosses this interface.
 *    A NULL handle (context, batch, network, sampler) or a NULL output
 *    pointer of a create call is ENS_EINVAL, checked before any device
 *    call.
 *  - Host arrays passed in are COPIED before the call returns; the caller
 *    keeps ownership and may free them at once.
 *  - The library allocates no large device memory of its own: the caller
 *    asks ens_workspace_size() and binds a device buffer of at least that
 *    size with ens_bind_workspace() (the buffer is BORROWED: it must stay
 *    alive and untouched until ens_destroy or a re-bind).  Only a few
 *    hundred bytes of per-context bookkeeping are allocated internally.
 *  - Device pointers given to ens_apply are borrowed for the call.
 *  - Layouts are row-major with samples fastest: an ensemble block is
 *    [rows][S] on the host and [rows][S_pad] on the device, S_pad >= S
 *    (query ens_info); dof index = 3*node + component (x, y, z).  Nodes and
 *    elements are numbered as the caller gave them in ens_set_mesh at every
 *    entry point; the library reorders them internally for locality (a
 *    recursive coordinate bisection into compact patches of <= 64 nodes).
 *  - Work is enqueued on the stream given to ens_step / ens_apply (a
 *    hipStream_t; NULL = the legacy default stream).  Set-up calls and
 *    read-backs synchronize.
 *  - Calls on one context are not thread-safe.  Distinct contexts are
 *    independent.
 */
#ifndef ENSFEM_H
#define ENSFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ens_ctx ens_ctx;

enum {
  ENS_OK = 0,
  ENS_EINVAL = -1,      /* bad argument: size, index, value range, NaN      */
  ENS_ESTATE = -2,      /* call out of order (missing mesh / ensemble / ...) */
  ENS_EWORKSPACE = -3,  /* workspace unbound or smaller than required       */
  ENS_EDEVICE = -4,     /* HIP runtime failure                               */
  ENS_EUNSTABLE = -5,   /* dt above the element-eigenvalue stability bound   */
  ENS_ENONFINITE = -6,  /* NaN / Inf found in the state by the watchdog      */
  ENS_EUNSUPPORTED = -7 /* option combination not implemented               */
};

/* precision of the stiffness apply */
enum { ENS_F64 = 0, ENS_F32 = 1 };
/* displacement state:
 *   F64        two-level (u_n, u_{n-1}) in FP64
 *   F32_KAHAN  velocity form (u, v) in FP32 with a Kahan-compensated
 *              u <- u + dt v (compensation term kept per dof)
 *   F32        velocity form in plain FP32 (shows what compensation buys) */
enum { ENS_STATE_F64 = 0, ENS_STATE_F32_KAHAN = 1, ENS_STATE_F32 = 2 };
/* apply kernel variant:
 *   NODE_GATHER  per-sample stiffness: each node gathers its incident
 *                elements' (E h)_{e,s} Khat_e rows (element-by-element,
 *                assembly-free, Sec. 2.4)
 *   CSR_SHARED   one stiffness for all samples ((E h)_{e,s} = (E h)_e):
 *                K assembled once into 3x3 block rows, applied as a
 *                sparse-matrix times ensemble-block product (the CSR
 *                product with 9 n_s entries per block of Sec. 2.3)
 *   AUTO         CSR_SHARED when every (E h) row is constant, else
 *                NODE_GATHER (ens_info reports the one in use) */
enum { ENS_VARIANT_AUTO = 0, ENS_VARIANT_NODE_GATHER = 1, ENS_VARIANT_CSR_SHARED = 3 };
/* load time factor g(t):  STEP g = 1;  RAMP_SINE g = sin(pi t / (2 t_ramp))
 * for t < t_ramp, else 1 (sine ramp of Sec. 3.1.2);  PULSATILE = RAMP_SINE
 * times (1 + amp sin(2 pi t / period)). */
enum { ENS_LOAD_STEP = 0, ENS_LOAD_RAMP_SINE = 1, ENS_LOAD_PULSATILE = 2 };
typedef struct {
  int32_t kind;
  double t_ramp;
  double amp;
  double period;
} ens_schedule;
/* quantities of interest */
enum { ENS_QOI_PEAK_RADIAL = 1, ENS_QOI_STRESS = 2 };
/* Wall-stress components in the cylindrical frame (ens_stress). */
enum { ENS_STRESS_THETA_THETA = 0, ENS_STRESS_Z_Z = 1, ENS_STRESS_THETA_Z = 2, ENS_STRESS_R_Z = 3 };

typedef struct {
  int64_t n_nodes, n_el, n_dof;
  int32_t S, S_pad, sample_block;
  int32_t apply_prec, state_prec, variant;
  int32_t shared_stiffness; /* 1 when every (E h) row is constant over samples */
  int64_t steps_done;
  double dt;                /* 0 until the first ens_step */
  size_t workspace_bytes;
} ens_info_t;

/* Lifetime.  ENS_EDEVICE if the HIP device cannot be selected. */
int32_t ens_create(int32_t device, ens_ctx** out);
int32_t ens_destroy(ens_ctx* ctx);
const char* ens_last_error(const ens_ctx* ctx);
int32_t ens_info(ens_ctx* ctx, ens_info_t* out);

/* Wall mesh (Sec. 2.2.1): xyz[n_nodes*3] node coordinates, tri[n_el*3]
 * node indices (counter-clockwise seen from outside), fixed_dof[n_nodes*3]
 * 1 = clamped (held at zero, its load ignored), radial[n_nodes*3] unit
 * outward radial direction per node (QoI, Sec. 2.2.3 local frame).
 * ENS_EINVAL for an index out of range, a degenerate triangle or a radial
 * vector that is not unit length (|1 - |r|| > 1e-6). */
int32_t ens_set_mesh(ens_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_el,
                     const int32_t* tri, const uint8_t* fixed_dof, const double* radial);

/* Material (Sec. 2.2.1 constitutive matrix; Sec. 2.3 damping C = alpha M):
 * 0 <= nu < 0.5, shear_k >= 0, rho > 0 (g/cm^3), alpha >= 0 (1/s). */
int32_t ens_set_material(ens_ctx* ctx, double nu, double shear_k, double rho, double alpha);

/* Mass scaling (Sec. 1: raising the critical step): for dt_target > 0 the
 * density of every element and sample whose eigenvalue bound
 * 3 E lambda_max(Khat_e) / (rho A_e) exceeds (2 / dt_target)^2 is multiplied
 * by that bound times dt_target^2 / 4, so ens_cfl_dt(ctx, 1.0) >= dt_target;
 * the lumped masses and the stability bound use the scaled densities.  0
 * (the default) turns it off.  Drops the workspace binding (re-bind).
 * ENS_EINVAL for a negative or non-finite dt_target. */
int32_t ens_set_mass_scaling(ens_ctx* ctx, double dt_target);

/* Explicit viscous force (Sec. 2.3): f_v = -c_d du/dt is added to the load,
 * with du/dt at t_n taken as (u_n - u_{n-1}) / dt so the step stays
 * explicit (and as v_0 in the starter); one coefficient c_d >= 0 for every
 * free dof, default 0.  The step's stability needs (omega dt)^2 < 4 -
 * 2 c_d dt / m per mode and node mass m, so c_d dt / m should stay well
 * below 1; the stability check of ens_step does not include this term.
 * Resets the state (call ens_init_state again).  ENS_EINVAL for a negative
 * or non-finite c_d. */
int32_t ens_set_viscous(ens_ctx* ctx, double c_d);

/* Geometry update with selective stiffness refresh (Sec. 2.3): for every > 0
 * each sample's element matrices are evaluated on its own moved geometry
 * x + u_m, where u_m is that sample's displacement at the last refresh
 * (steps m = every, 2 every, ...; the first interval is the linear model,
 * u_0 = 0).  The internal force is carried incrementally:
 * R_n = R_m + K(x + u_m) (u_n - u_m), and a refresh at step m first moves
 * the base to R_m = R_m' + K(x + u_m') (u_m - u_m'), so the force does not
 * jump when the matrix changes.  Masses, the load and the stability bound
 * stay those of the reference geometry; the starter, ens_stress and
 * ens_apply use the reference geometry.  Needs the FP64 state
 * (ENS_STATE_F64) and no energy records: ens_step returns ENS_EUNSUPPORTED
 * otherwise, and ens_save / ens_load / ens_batch_create refuse such a
 * context.  0 (the default) turns it off.  Switching it on or off drops the
 * workspace binding (the snapshot u_m and the base R_m take 48 B per node
 * and padded sample); any change resets the state (the same value again
 * changes nothing).  ENS_EINVAL for every < 0. */
int32_t ens_set_geometry_refresh(ens_ctx* ctx, int32_t every);

/* Ensemble fields: eh[n_el*S] = (E h)_{e,s} (element-wise product of
 * modulus and thickness, the scalar that multiplies the reference element
 * stiffness, Sec. 2.2.1 / Sec. 2.4) and h[n_el*S] thickness (lumped mass
 * rho h A / 3 per node, Sec. 2.3).  ENS_EINVAL if S < 1 or any value is not
 * finite and positive. */
int32_t ens_set_ensemble(ens_ctx* ctx, int32_t S, const double* eh, const double* h);

/* Load: F[n_nodes*3] nodal traction force (shared by all samples) and its
 * time factor; f_n = g(n dt) F. */
int32_t ens_set_load(ens_ctx* ctx, const double* F, ens_schedule sched);

/* Precision / variant / outputs.  qoi_mask: ENS_QOI_PEAK_RADIAL to track
 * q_{i,s} = max_n e_r,i . u_{i,s}(t_n); ENS_QOI_STRESS to reserve the
 * scratch of ens_stress / ens_stress_bands.  energy_every > 0 records the
 * discrete energy 1/2 v^T M v + 1/2 u_{n+1}^T K u_n per sample at steps
 * n with n % energy_every == 0 (the most recent 4096 records are kept).
 * ENS_VARIANT_CSR_SHARED needs shared stiffness (ENS_EUNSUPPORTED at bind
 * otherwise). */
int32_t ens_configure(ens_ctx* ctx, int32_t apply_prec, int32_t state_prec, int32_t variant,
                      int32_t qoi_mask, int32_t energy_every);

/* Device workspace: size for the current mesh / ensemble / configuration,
 * then bind.  Binding uploads everything and runs the set-up kernels
 * (element matrices, lumped mass, stability bound).  ENS_EWORKSPACE if
 * bytes is below the required size or dptr is NULL or not 256-B aligned. */
int32_t ens_workspace_size(ens_ctx* ctx, size_t* bytes);
int32_t ens_bind_workspace(ens_ctx* ctx, void* dptr, size_t bytes);

/* Largest stable step times `safety`: dt = safety * 2 / omega_hat with
 * omega_hat^2 = max_{e,s} 3 E_{e,s} lambda_max(Khat_e) / (rho A_e), an upper
 * bound on the assembled pencil's largest eigenvalue. */
int32_t ens_cfl_dt(ens_ctx* ctx, double safety, double* dt_out);

/* Initial state u0, v0 [n_nodes*3*S] (NULL = zero).  Resets the step count,
 * the QoI and the energy log.  The Taylor starter u_{-1} is formed at the
 * first ens_step, when dt is known. */
int32_t ens_init_state(ens_ctx* ctx, const double* u0, const double* v0);

/* Enqueue n_steps explicit steps of size dt on `stream` (hipStream_t); runs
 * without energy records or geometry refresh go in replays of a captured
 * graph of 64 steps (same kernels, same results as direct launches).  dt
 * is fixed by the first call after ens_init_state (which also forms the
 * starter, even with n_steps = 0); later calls must pass the same value
 * (ENS_EINVAL otherwise).  ENS_EUNSTABLE if dt exceeds the
 * stability bound (2 / omega_hat) unless `force` is nonzero.  ENS_ESTATE if
 * mesh, ensemble, load, state or workspace is missing. */
int32_t ens_step(ens_ctx* ctx, int64_t n_steps, double dt, int32_t force, void* stream);

/* Wait for the context's work; ENS_ENONFINITE if the state holds NaN/Inf.
 * With energy records on (energy_every > 0) every record also runs the
 * energy watchdog: the discrete energy of a stable central-difference step
 * is at least (1 - s^2) times its kinetic part, s = dt omega_hat / 2 from
 * the stability bound (capped at 0.999 for a forced step), in any state; a
 * record that breaks this marks the run unstable and ens_sync returns
 * ENS_EUNSTABLE (until ens_init_state or ens_load).  Nothing is checked
 * without energy records. */
int32_t ens_sync(ens_ctx* ctx);

/* Read-backs into caller-owned host buffers (synchronizing):
 * state u_n [n_nodes*3*S]; QoI [n_nodes*S]; energy records (up to
 * max_records most recent, chronological): steps_out[k], e_out[k*S];
 * per-node ensemble mean and unbiased variance of the QoI [n_nodes]. */
int32_t ens_read_state(ens_ctx* ctx, double* u);
int32_t ens_read_qoi(ens_ctx* ctx, int32_t kind, double* out);
int32_t ens_read_energy(ens_ctx* ctx, int64_t max_records, int64_t* steps_out, double* e_out,
                        int64_t* n_out);
int32_t ens_moments(ens_ctx* ctx, double* mean, double* var);

/* Allocation-free ens_moments, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same inputs, outputs and results as ens_moments (the
 * same kernel and summation order: bitwise equal); its device staging lives
 * in a fixed 16 MiB scratch array that the library holds on each GPU it runs
 * on until the process ends, so it takes at most 1,048,576 nodes
 * (ENS_EINVAL with a message beyond that; ens_moments has no such limit).
 * The call allocates nothing (no hipMalloc / hipFree, no host buffers).
 * Every call on a GPU shares that GPU's scratch and leaves its contents
 * behind: calls that overlap on one GPU (from several threads or contexts)
 * race and must be serialised by the caller.  Synchronizing. */
int32_t ens_moments_noalloc(ens_ctx* ctx, double* mean, double* var);

/* Wall stress of the current state in the local cylindrical frame (Sec.
 * 2.3, fluid-structure coupling): per element and sample, the local strains
 * of Sec. 2.2.1 (B times the element's nodal displacements in its frame),
 * stresses sigma = C eps with E = (E h)/h and sigma_zz = 0, taken to the
 * frame r = the element's unit normal, z = axial[e] (the centreline tangent
 * at the element, caller's element order, [n_el*3] host) with its normal
 * part removed and normalised, theta = r x z.  component: one of
 * ENS_STRESS_*; out [n_el*S] host.  Needs ENS_QOI_STRESS in ens_configure
 * (it sizes a scratch region of n_el*(S_pad+6) doubles in the workspace);
 * ENS_ESTATE otherwise or without a state, ENS_EINVAL for a zero or
 * non-finite tangent or one parallel to its element's normal.
 * Synchronizing. */
int32_t ens_stress(ens_ctx* ctx, const double* axial, int32_t component, double* out);
/* Ensemble bands of one stress component per element: mean over the S
 * samples and the p_lo / p_hi quantiles (linear interpolation between order
 * statistics at p (S - 1)), host arrays [n_el] in the caller's element
 * order.  S <= 4096 (ENS_EUNSUPPORTED otherwise); levels in [0, 1]. */
int32_t ens_stress_bands(ens_ctx* ctx, const double* axial, int32_t component, double p_lo, double p_hi,
                         double* mean, double* lo, double* hi);

/* Stand-alone stiffness apply R = K(E h)_s U on device buffers of
 * [n_nodes*3][S_pad] in `prec` (ENS_F64: double, ENS_F32: float), using
 * the bound context's mesh and fields, no boundary conditions. */
int32_t ens_apply(ens_ctx* ctx, int32_t prec, const void* U_dev, void* R_dev, void* stream);

/* Performance tuning of the step kernels (no effect on results beyond
 * rounding order): sample_block in {0 = auto, 8, 16, 32, 64, 128, 256}
 * samples per node per workgroup pass (128 and 256 give each of 64 lanes 2
 * or 4 consecutive samples), sb_inner = 1 orders workgroups
 * sample-block-fastest.  A
 * change of the padded width drops the workspace binding (re-bind). */
int32_t ens_set_tuning(ens_ctx* ctx, int32_t sample_block, int32_t sb_inner);

/* Checkpoint of the time-stepping state (state arrays, step count, dt,
 * QoI).  ens_save with host == NULL writes the size to *bytes.  The blob is
 * opaque: rows are stored in the library's internal node order, so it
 * restores only into a context given the same mesh and sample count. */
int32_t ens_save(ens_ctx* ctx, void* host, size_t* bytes);
int32_t ens_load(ens_ctx* ctx, const void* host, size_t bytes);

/* ---- Batching: many meshes per launch ---------------------------------
 * A batch steps several contexts together (one launch per time step, or
 * one per lane class, whose workgroups each take one (mesh, node tile,
 * sample block) tile of a list; the step loop is captured in a hipGraph and
 * replayed).  Each
 * context keeps its own mesh, fields, load, dt and state and stays usable
 * on its own between batch calls.  Requirements (ENS_EINVAL otherwise, the
 * message on the offending context): bound workspaces on one device, the
 * same apply / state precision and QoI setting, node-gather variant, no
 * energy records, padded width S_pad a multiple of 32 (ens_set_tuning with
 * a sample block of 32 or more before binding).  The batch owns
 * small device tables (tiles, per-mesh arguments) and a stream of its own;
 * ens_batch_step orders itself after prior work on `stream` and makes
 * `stream` wait for it. */
typedef struct ens_batch ens_batch;
typedef struct {
  int32_t n_meshes, n_tiles;
  int32_t samples_per_lane; /* 64 lanes x up to this many samples per tile */
  int32_t tile_nodes;       /* nodes per tile (4: one per wave)          */
  int32_t grid;             /* 0: one workgroup per tile (the only form) */
  int32_t graph_steps;      /* steps per captured graph                  */
  int32_t launches_per_step; /* 1, or 2 when full and tail blocks are
                                launched separately                      */
  double tuned_ms_per_step; /* best autotuner trial, 0 before autotune   */
  int32_t concurrent_tails;  /* 1: the tail launches run on a second
                                stream beside the full blocks          */
  int32_t reserved_;
} ens_batch_info_t;

int32_t ens_batch_create(ens_ctx** ctxs, int32_t n, ens_batch** out);
int32_t ens_batch_destroy(ens_batch* b);
const char* ens_batch_last_error(const ens_batch* b);
int32_t ens_batch_info(ens_batch* b, ens_batch_info_t* out);
/* n_steps steps of every mesh.  Every context must have its state set and
 * dt fixed (ens_init_state, then ens_step(ctx, 0, dt, ...)).  Results are
 * bitwise those of stepping each context alone. */
int32_t ens_batch_step(ens_batch* b, int64_t n_steps, void* stream);
/* Times trial_steps steps for each candidate tiling and keeps the fastest:
 * samples per lane 1 or 2 (blocks of 64 or 128 samples; the samples left
 * at the end of a mesh, 64 or 32, form a tail block run at one sample per
 * lane; with 2 per lane, 96 left form one block on 48 lanes among the full
 * ones) and, with 2, the tail blocks in the same launch, in a second
 * launch per step, or in a second launch on a second stream.  Every tiling
 * has one workgroup per tile of 4 nodes.
 * The trial steps ADVANCE every context's state: re-init the states
 * afterwards to restart from the initial condition. */
int32_t ens_batch_autotune(ens_batch* b, int32_t trial_steps);
/* Sets the tiling without timing trials: samples_per_lane 1 or 2; split 1
 * runs the tail blocks in a launch of their own (one sample per lane), 2
 * the same on a second stream of the batch beside the full blocks (a
 * sample column's steps depend only on that column), 0 in the same launch.
 * ENS_EINVAL for other values.  Results do not depend on the tiling. */
int32_t ens_batch_set_tiling(ens_batch* b, int32_t samples_per_lane, int32_t split);

#ifdef __cplusplus
}
#endif

#endif /* ENSFEM_H */
