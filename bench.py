"""Benchmark of the explicit ensemble wall step on one MI355X.

Workload: straight clamped cylinder, 400 x 500 nodes (200,000 nodes, 399,200
linear triangles, 600,000 dof), S = 256 lognormal Matern (E, h) samples,
steady internal pressure 1.33e5 dyn/cm^2, Rayleigh alpha = 50 1/s, dt = 0.9 x
the element-eigenvalue bound.  One "step" = one explicit time step of the
whole hot path (stiffness apply + central-difference update + load + peak
radial QoI) for all 256 samples.

Prints ONE JSON line: throughput in dof*sample*steps/s (inputs resident in
HBM), the roofline of the fused step kernel (algorithmic bytes per launch /
its average duration from HIP events on the launch stream) and the CPU
oracle timed on a bounded sample on the host.

    python bench.py [--steps K] [--warmup W] [--apply f32|f64] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import math
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_kernel_bytes(n_nodes: int, n_el: int, S: int, apply_f32: bool, state: str = "f64") -> dict:
    """Algorithmic HBM bytes of one fused step launch.  State traffic per
    dof and sample: FP64 state reads u_n and u_{n-1} and writes u_{n+1}
    (3 x 8 B); FP32-Kahan reads and writes u, its compensation and the
    velocity (6 x 4 B); plain FP32 reads and writes u and the velocity
    (4 x 4 B).  Plus (E h) per element and sample and 1/m per node and
    sample (4 B in the FP32 apply, 8 B in FP64), the rising bit of the
    running peak read and written (1/8 B each per node and sample; the
    stored peak itself is only touched at local maxima of the radial
    displacement, so it is not counted), and the per-mesh arrays read once
    per launch
    (adjacency and 3x6 stiffness blocks, load, radial directions, clamp
    bits)."""
    w = 4 if apply_f32 else 8
    state_b = {"f64": 24, "f32_kahan": 24, "f32": 16}[state]
    n_dof = 3 * n_nodes
    n_adj = 3 * n_el
    per_sample = n_dof * state_b + n_el * w + n_nodes * w + n_nodes * 0.25
    per_mesh = n_adj * (18 * w + 4 + 8) + (n_nodes + 1) * 4 + n_nodes * (24 + 24 + 1)
    return dict(total=int(per_sample * S + per_mesh), per_sample=per_sample, per_mesh=per_mesh)


def source_hash() -> str:
    """Hash of what decides the step kernels' memory traffic: the kernel
    sources, the host code that picks their launch shapes, the node
    ordering and the batch tile list, and the compiler flags."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2101_09059_amd")
    for f in ("csrc/step.hip", "csrc/internal.h", "csrc/api.hip", "build.py"):
        with open(os.path.join(pkg, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, variant: str, launches_bytes: int):
    """(FETCH_SIZE + WRITE_SIZE traffic per launch scaled by the copy
    calibration, the same with reads counted by request size) from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        rec = d.get(f"{workload}:{variant}")
        if not rec or rec.get("source_hash") != source_hash():
            return None
        return int(rec["bytes_per_launch"]), rec.get("bytes_per_launch_by_request_size")
    except Exception:
        return None


_BARRIER = None


def _pool_init(barrier):
    global _BARRIER
    _BARRIER = barrier


def _oracle_column(task):
    """Worker of the all-cores CPU baseline: the oracle on one sample column
    (own element matrices and CSR assembly), stepping started together with
    the other workers; returns the wall-clock interval of its stepping."""
    xyz, tri, fixed, radial, F, eh_col, h_col, cfg, dt, steps = task
    from oracle import element, stepper
    kh, A, _ = element.reference_stiffness(xyz, tri, cfg["nu"], cfg["shear_k"])
    _BARRIER.wait(timeout=120)
    t0 = time.time()
    stepper.run_ensemble(tri, kh, A, eh_col[:, None], h_col[:, None], cfg["rho"], F, fixed, radial, dt, steps,
                         cfg["alpha"], lambda t: 1.0)
    return t0, time.time()


def _oracle_c3_column(task):
    """Worker of the precision-form check: the oracle on one sample column of
    the full curved tube (its own element matrices, per-sample CSR stiffness
    and lumped mass, eq. dynamicsCD step by step) for n_steps steps, with the
    step size from the oracle's element bound over the whole ensemble
    (ratio = max over samples of E = (E h) / h per element).  Returns u, q and
    the step size it used."""
    eh_col, h_col, ratio, n_steps = task
    from paper_2101_09059_amd import inputs
    from oracle import cfl, element, stepper
    c = inputs.CONFIGS["c3_curved"]
    m = inputs.curved_tube(c["n_theta"], c["n_z"])
    F = inputs.traction_load(m, c["p0"], axial_taper=c["axial_taper"], shear_frac=c["shear_frac"], seed=c["seed"])
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, c["nu"], c["shear_k"])
    dt = cfl.stable_dt(kh, A, ratio[:, None], np.ones((m.n_el, 1)), c["rho"], c["safety"])
    g = lambda t: stepper.load_factor(c["ramp"], t, c["T_ramp"], c["period"], c["pulse_amp"])
    r = stepper.run_ensemble(m.tri, kh, A, eh_col[:, None], h_col[:, None], c["rho"], F, m.fixed, m.radial, dt,
                             n_steps, c["alpha"], g)
    return r["u"][:, 0], r["q"][:, 0], dt


def cpu_baseline(mesh, eh, h, F, cfg, dt, budget_s: float = 12.0) -> dict:
    """The oracle as it stands (per-sample CSR assembly + one SpMV and update
    per step) on a bounded sample of the same workload: one process, then one
    process per host core (up to 16) with one sample column each, all
    stepping at once (wall clock from the first start to the last end)."""
    from oracle import element, stepper
    t0 = time.perf_counter()
    kh, A, _ = element.reference_stiffness(mesh.xyz, mesh.tri, cfg["nu"], cfg["shear_k"])
    t_el = time.perf_counter() - t0
    steps, samples = 40, [0]
    t0 = time.perf_counter()
    stepper.run_ensemble(mesh.tri, kh, A, eh, h, cfg["rho"], F, mesh.fixed, mesh.radial, dt, steps,
                         cfg["alpha"], lambda t: 1.0, samples=samples)
    t1 = time.perf_counter() - t0
    # grow the sample within the budget
    more = max(0, int((budget_s - t_el - t1) / max(t1, 1e-3)))
    if more:
        extra = list(range(1, 1 + min(more, 15)))
        t0 = time.perf_counter()
        stepper.run_ensemble(mesh.tri, kh, A, eh, h, cfg["rho"], F, mesh.fixed, mesh.radial, dt, steps,
                             cfg["alpha"], lambda t: 1.0, samples=extra)
        t1 += time.perf_counter() - t0
        samples += extra
    one = mesh.n_dof * len(samples) * steps / t1
    del kh, A
    workers = max(1, min(16, os.cpu_count() or 1))
    note = ""
    try:
        import multiprocessing as mp
        ctx = mp.get_context("spawn")
        barrier = ctx.Barrier(workers)
        tasks = [(mesh.xyz, mesh.tri, mesh.fixed, mesh.radial, F, np.ascontiguousarray(eh[:, s]),
                  np.ascontiguousarray(h[:, s]), cfg, dt, steps) for s in range(workers)]
        with ctx.Pool(workers, initializer=_pool_init, initargs=(barrier,)) as pool:
            spans = pool.map_async(_oracle_column, tasks, chunksize=1).get(timeout=240)
        wall = max(b for _, b in spans) - min(a for a, _ in spans)
        value, cores = mesh.n_dof * workers * steps / wall, workers
        note = (f"; all cores: {workers} processes x 1 sample column x {steps} steps, "
                f"{wall:.1f} s wall from the first start to the last end")
    except Exception as ex:  # report the one-process figure, say why
        value, cores = one, 1
        note = f"; the {workers}-process run failed ({type(ex).__name__}: {ex}), one-process figure reported"
    return {"value": value, "unit": "dof*sample*steps/s", "cores": cores, "kind": "oracle",
            "value_one_core": one,
            "sample": f"one process: {len(samples)} sample columns x {steps} steps of the same {mesh.n_dof:,}-dof mesh "
                      f"(per-sample CSR assembly + SpMV + update), {t1:.1f} s timed, element matrices "
                      f"({t_el:.1f} s) excluded{note}; host nproc={os.cpu_count()}"}


def run_batch_config(args, torch):
    """Batching form: 16 seeded tubes of uneven size and width, FP32 apply /
    FP64 state, one launch per step over all meshes (graph-captured loop,
    autotuned tiling), against stepping the meshes one after another (their
    own contexts, each with the library's own sample-block choice).  Each
    batch member is padded to a multiple of 32 samples (64 where S is one);
    the byte model counts the S real samples only."""
    from paper_2101_09059_amd import ensfem, inputs
    cfg = inputs.CONFIGS["c4_batch"]
    specs = inputs.tube_batch_specs(cfg["seed"], cfg["count"])
    t0 = time.perf_counter()
    members, solo, work_per_step, bytes_per_step, pad_per_step = [], [], 0, 0, 0
    for i, sp in enumerate(specs):
        m = inputs.cylinder(sp["R"], sp["L"], sp["n_theta"], sp["n_z"])
        eh, h = inputs.lognormal_fields(m, sp["S"], cfg["seed"] * 1000 + i)
        F = inputs.traction_load(m, cfg["p0"])
        kw = dict(nu=cfg["nu"], shear_k=cfg["shear_k"], rho=cfg["rho"], alpha=cfg["alpha"], apply_prec=ensfem.F32)
        ens = ensfem.setup_case(m, eh, h, F, sample_block=64 if sp["S"] % 64 == 0 else 32, **kw)
        one = ensfem.setup_case(m, eh, h, F, **kw)
        dt = ens.cfl_dt(cfg["safety"])
        for e in (ens, one):
            e.init_state()
            e.step(0, dt)
        members.append((ens, dt))
        solo.append((one, dt))
        work_per_step += m.n_dof * sp["S"]
        bytes_per_step += step_kernel_bytes(m.n_nodes, m.n_el, sp["S"], True)["total"]
        pad_per_step += m.n_nodes * (ens.info()["S_pad"] - sp["S"])
        del eh, h
        log(f"mesh {i}: {m.n_nodes} nodes, S={sp['S']} ready ({time.perf_counter() - t0:.0f} s)")
    batch = ensfem.Batch([e for e, _ in members])
    batch.autotune(5)
    info = batch.info()
    log(f"autotuned: {info}")
    stream = torch.cuda.current_stream()
    for e, dt in members:  # restart from rest after the tuning trials
        e.init_state()
        e.step(0, dt)
    batch.step(args.warmup, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    batch.step(args.steps, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # the same meshes stepped one after another (one launch per mesh per step)
    seq_steps = max(10, args.steps // 10)
    e0.record(stream)
    for _ in range(seq_steps):
        for e, dt in solo:
            e.step(1, dt, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1) / seq_steps
    for e, _ in members + solo:
        e.sync()
    batch.close()
    for e, _ in members + solo:
        e.close()
    per = ms / args.steps
    achieved = bytes_per_step / (per * 1e-3) / 1e9
    traffic = measured_traffic("c4_batch", "batch_step_f32apply_f64state", bytes_per_step)
    out = {
        "metric": "ensemble dof*sample*steps/s", "value": work_per_step / (per * 1e-3),
        "unit": "dof*sample*steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": per, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 apply / f64 state", "data": "synthetic",
        "config": {"workload": "batch of 16 seeded straight tubes (5k-400k nodes log-uniform, R 0.3-1.5 cm, "
                               "L 5-25 cm, S 32-512), steady pressure, alpha=50, per-mesh dt",
                   "dof_samples_per_step": work_per_step,
                   "padding_node_samples_per_step": pad_per_step, "batch": info, "parallelism": "single GPU"},
        "ms_per_step_one_mesh_at_a_time": ms_seq,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic[0] if traffic else None,
                     "kernel": "k_batch_step (full-block and tail launches of one step)",
                     "algorithmic_bytes_per_launch": bytes_per_step},
    }
    print(json.dumps(out), flush=True)


def run_surrogate_kernels(args, torch):
    """The learned form's kernels at full size on random data: the network
    128 -> 3 x 1024 GELU -> 200,000 (BF16 MFMA, FP32 accumulate), one Adam
    training step on a batch of 256, a forward pass of 256 rows, and the
    per-output sums over 65,536 rows."""
    from paper_2101_09059_amd import ensfem
    sizes = [128, 1024, 1024, 1024, 200000]
    net = ensfem.Surrogate(128, 1024, 3, 200000, 256)
    rng = np.random.default_rng(9)
    net.set_params((0.02 * rng.standard_normal(net.n_params)).astype(np.float32))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)
    X = torch.randn(256, 128, device="cuda", generator=gen)
    T = torch.randn(256, 200000, device="cuda", generator=gen)
    Y = torch.empty(256, 200000, device="cuda")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, n):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    n = max(1, min(args.steps, 50))
    ms_train = timed(lambda: net.train_step(X, T, 1e-5), n)
    ms_fwd = timed(lambda: net.forward(X, out=Y), n)
    Xl = torch.randn(65536, 128, device="cuda", generator=gen)
    net.moments(Xl)
    t0 = time.perf_counter()
    net.moments(Xl)
    s_mom = time.perf_counter() - t0
    flops_fwd = 2.0 * 256 * sum(a * b for a, b in zip(sizes[:-1], sizes[1:]))
    # at 256 rows the pass is bound by HBM: BF16 weights read once, FP32
    # biases, the input and the FP32 output (171 flop/B, below the BF16
    # ridge of ~310 flop/B)
    bytes_fwd = 2 * (net.n_params - sum(sizes[1:])) + 4 * sum(sizes[1:]) + 4 * 256 * (sizes[0] + sizes[-1])
    achieved = bytes_fwd / (ms_fwd * 1e-3) / 1e9
    out = {"metric": "surrogate kernels: Adam training step (batch 256)", "value": ms_train, "unit": "ms",
           "n_gpus": 1, "steps": n, "higher_is_better": False, "data": "synthetic (random parameters and data)",
           "dtype": "bf16 mfma / fp32 accumulate",
           "config": {"workload": "MLP 128 -> 3 x 1024 GELU -> 200,000 (207,231,296 parameters)"},
           "forward_ms_batch_256": ms_fwd, "moments_65536_rows_s": s_mom,
           "forward_tflops": flops_fwd / (ms_fwd * 1e-3) / 1e12,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "forward pass (k_gemm)",
                        "algorithmic_bytes_per_pass": bytes_fwd}}
    print(json.dumps(out), flush=True)


def variance_se_rows(q: np.ndarray) -> np.ndarray:
    """Per row, the standard error of the sample variance of the columns of
    q without assuming normality: sqrt((m4 - m2^2) / N) (fourth central
    moment m4), the estimate's spread for heavy-tailed samples."""
    N = q.shape[1]
    d = q - q.mean(axis=1, keepdims=True)
    m2 = (d * d).mean(axis=1)
    m4 = (d ** 4).mean(axis=1)
    return np.sqrt(np.maximum(m4 - m2 * m2, 0.0) / N)


def cv_variance_bootstrap_se(qH, qL, sumL, sumsqL, M, n_boot=100, n_nodes=4096, seed=1):
    """Relative standard error of the control-variate variance estimate,
    from resampling the N high-fidelity pairs (the M network draws held
    fixed): on a random subset of varying nodes, the norm of the per-node
    spread over the replicates divided by the norm of the estimate."""
    rng = np.random.default_rng(seed)
    act = np.flatnonzero(qH.var(axis=1) > 0)
    nodes = rng.choice(act, size=min(n_nodes, act.size), replace=False)
    H, L = qH[nodes], qL[nodes]
    mL = (sumL[nodes] / M, sumsqL[nodes] / M)
    N = H.shape[1]

    def cv_var(h0, l0):
        est = []
        for k, (h, l) in enumerate(((h0, l0), (h0 * h0, l0 * l0))):
            mh, ml = h.mean(1), l.mean(1)
            cov = ((h - mh[:, None]) * (l - ml[:, None])).sum(1) / (N - 1)
            vl = l.var(1, ddof=1)
            beta = np.where(vl > 0, cov / np.where(vl > 0, vl, 1.0), 0.0)
            est.append(mh - beta * (ml - mL[k]))
        return est[1] - est[0] ** 2

    base = cv_var(H, L)
    reps = np.empty((n_boot, nodes.size))
    for b in range(n_boot):
        idx = rng.integers(0, N, N)
        reps[b] = cv_var(H[:, idx], L[:, idx])
    return float(np.linalg.norm(reps.std(axis=0)) / np.linalg.norm(base))


def run_learned_config(args, torch):
    """Learned form at full size: 200k-node cylinder, 64 + 64 KL inputs,
    MLP 128 -> 3 x 1024 (GELU) -> 200,000, trained on 4,096 solver samples
    (80 % fit, 10 % early-stopping validation, 10 % held out; AdamW);
    control variate from N = 1,024 plain samples and 65,536 network draws,
    judged against a plain reference of 8,192 fresh samples."""
    from paper_2101_09059_amd import inputs, learned
    c = inputs.CONFIGS["c5_learned"]
    sd = c["seeds"]
    mesh = inputs.cylinder(c["R"], c["L"], c["n_theta"], c["n_z"])
    prob = learned.Problem(mesh, c, c["n_modes"])
    log(f"KL basis: {c['n_modes']} modes per field capture {prob.captured:.3f} of the variance")
    S = 256

    def solve_many(seed, n):
        X = learned.draw_xi(seed, n, c["n_modes"])
        qs = []
        for i in range(0, n, S):
            qs.append(prob.solve(X[i:i + S], progress=lambda m: log(f"    batch {i // S}: {m}")))
            log(f"  solved {i + S}/{n} (seed {seed}), solver time {prob.solve_seconds:.0f} s")
        return X, np.concatenate(qs, axis=1)

    t_data0 = prob.solve_seconds
    Xtr, Qtr = solve_many(sd["train"], c["n_train"])
    t_data = prob.solve_seconds - t_data0
    net = learned.Network(2 * c["n_modes"], c["width"], c["n_hidden"], mesh.n_nodes, seed=sd["init"], max_batch=256)
    Qs = np.ascontiguousarray(Qtr.T)  # [samples][nodes]
    del Qtr
    rmse, hist = net.fit(Xtr, Qs, epochs=c["epochs"], batch=c["batch"], lr=c["lr"], seed=sd["init"] + 1,
                         val=c["val"], weight_decay=c["weight_decay"], progress=log)
    del Qs
    log(f"trained in {net.train_seconds:.1f} s: held-out rel RMSE {rmse:.4f}, loss {hist[0]:.3e} -> {hist[-1]:.3e}, "
        f"kept epoch {net.best_epoch}")
    t0 = prob.solve_seconds
    Xh, qH = solve_many(sd["hf"], c["n_hf"])  # in ensembles of 256, like every other solve
    t_hf = prob.solve_seconds - t0
    pm, pv = qH.mean(axis=1), qH.var(axis=1, ddof=1)  # the plain N-sample statistics
    qL = net.predict(Xh).T
    Xl = learned.draw_xi(sd["lf"], c["n_lf"], c["n_modes"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sumL, sumsqL = net.moment_sums(Xl)
    t_lf = time.perf_counter() - t0
    est = learned.estimate(qH, pm, pv, qL, sumL, sumsqL, c["n_lf"], rmse)
    vr_boot = learned.bootstrap_variance_ratio(qH, qL, sumL, c["n_lf"])
    log(f"median rho {est['rho_median']:.4f}, control variate used: {est['used_cv']}, "
        f"bootstrap variance reduction x{vr_boot:.1f}")
    _, qR = solve_many(sd["ref"], c["n_ref"])
    act = qR.var(axis=1) > 0
    ref_m, ref_v = qR.mean(axis=1), qR.var(axis=1, ddof=1)
    Nr = qR.shape[1]
    rel = lambda a, b: float(np.linalg.norm(a[act] - b[act]) / np.linalg.norm(b[act]))
    se_mean = float(np.linalg.norm(np.sqrt(ref_v[act] / Nr)) / np.linalg.norm(ref_m[act]))
    se_var_normal = float(np.sqrt(2.0 / (Nr - 1)))
    # the QoI is heavy-tailed (lognormal fields): the reference variance's
    # own error from its fourth moments, aggregated like the error metric
    se_var = float(np.linalg.norm(variance_se_rows(qR[act])) / np.linalg.norm(ref_v[act]))
    se_var_cv = cv_variance_bootstrap_se(qH, qL, sumL, sumsqL, c["n_lf"]) if est["used_cv"] else None
    err_mean, err_var = rel(est["mean"], ref_m), rel(est["var"], ref_v)
    var_bound = max(0.01, 2.0 * se_var)
    N, M = c["n_hf"], c["n_lf"]
    ratio = 1.0 - est["rho"][act] ** 2 * M / (M + N)
    n_eq = N / float(np.median(ratio))
    t_per_sample = t_hf / N
    t_plain_eq = n_eq * t_per_sample
    t_cv = t_hf + t_lf + net.train_seconds
    out = {
        "metric": "surrogate-CV QoI rel.err and speedup", "value": t_plain_eq / t_cv,
        "unit": "speedup over the plain ensemble at equal variance (training data excluded)",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "bf16 mfma / fp32 accumulate",
        "config": {"workload": f"200k-node clamped cylinder, pulsatile pressure (ramp 0.02 s, peak over the "
                               f"window t in [0, 0.03 s]), 64+64 KL inputs, MLP 3x1024 GELU -> 200,000, 4,096 "
                               f"training solves, {N:,} high-fidelity + {M:,} low-fidelity, plain reference {Nr:,}"},
        "mean_rel_err_vs_reference": err_mean,
        "var_rel_err_vs_reference": err_var,
        "plain_N_mean_rel_err": rel(pm, ref_m), "plain_N_var_rel_err": rel(pv, ref_v),
        "reference_se_mean": se_mean, "reference_se_var": se_var, "reference_se_var_if_normal": se_var_normal,
        "cv_var_se_bootstrap": se_var_cv,
        "acceptance": {"mean_within_1pct": err_mean <= 0.01, "var_bound_max_1pct_2se_ref": var_bound,
                       "var_within_bound": err_var <= var_bound,
                       "var_z_vs_combined_se": err_var / float(np.hypot(se_var, se_var_cv or 0.0))},
        "used_control_variate": est["used_cv"], "rho_median": est["rho_median"],
        "heldout_rel_rmse": rmse, "kl_captured_variance": prob.captured, "kept_epoch": net.best_epoch,
        "equivalent_plain_samples": n_eq,
        "variance_reduction_predicted": float(1.0 / np.median(ratio)),
        "variance_reduction_bootstrap": vr_boot,
        "speedup_including_training_data": t_plain_eq / (t_cv + t_data),
        "seconds": {"training_data": t_data, "training": net.train_seconds, "high_fidelity_N": t_hf,
                    "network_M_draws": t_lf, "plain_equivalent": t_plain_eq},
        "n_params": net.net.n_params,
    }
    net.close()
    print(json.dumps(out), flush=True)


def run_precision_config(args, torch):
    """Precision form at full size: 1M-node curved tapered tube, S = 1,024,
    sine-ramped pulsatile pressure with axial taper and wall shear.
    Throughput of each precision mode at S = 1,024, and the error of each
    FP32 mode against the FP64 path over a longer run on the first sample
    columns (same mesh, fields and load)."""
    from paper_2101_09059_amd import ensfem, inputs
    cfg = inputs.CONFIGS["c3_curved"]
    t0 = time.perf_counter()
    mesh = inputs.curved_tube(cfg["n_theta"], cfg["n_z"])
    S = cfg["S"]
    eh, h = inputs.lognormal_fields_device(mesh, S, cfg["seed"], radius=0.9)
    F = inputs.traction_load(mesh, cfg["p0"], axial_taper=cfg["axial_taper"], shear_frac=cfg["shear_frac"],
                             seed=cfg["seed"])
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s: {mesh.n_nodes} nodes, {mesh.n_el} tri, S={S}")
    modes = [("f64", ensfem.F64, ensfem.STATE_F64, "f64"),
             ("f32_apply_f64_state", ensfem.F32, ensfem.STATE_F64, "f64"),
             ("f32_apply_kahan_f32_state", ensfem.F32, ensfem.STATE_F32_KAHAN, "f32_kahan"),
             ("f32", ensfem.F32, ensfem.STATE_F32, "f32")]

    def make(fields, hh, ap, st):
        return ensfem.setup_case(mesh, fields, hh, F, nu=cfg["nu"], shear_k=cfg["shear_k"], rho=cfg["rho"],
                                 alpha=cfg["alpha"], kind=ensfem.LOAD_PULSATILE, t_ramp=cfg["T_ramp"],
                                 amp=cfg["pulse_amp"], period=cfg["period"], apply_prec=ap, state_prec=st)

    steps = min(args.steps, 200)
    stream = torch.cuda.current_stream()
    thr = {}
    dt = None
    for name, ap, st, sb in modes:
        ens = make(eh, h, ap, st)
        dt = ens.cfl_dt(cfg["safety"])
        ens.init_state()
        ens.step(10, dt, stream=stream)
        ens.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ens.step(steps, dt, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ens.sync()
        S_pad = ens.info()["S_pad"]
        ens.close()
        del ens
        torch.cuda.empty_cache()
        b = step_kernel_bytes(mesh.n_nodes, mesh.n_el, S_pad, ap == ensfem.F32, sb)["total"]
        thr[name] = dict(ms_per_step=ms, value=mesh.n_dof * S / (ms * 1e-3), achieved_GBs=b / (ms * 1e-3) / 1e9)
        log(f"{name}: {ms:.3f} ms/step, {thr[name]['achieved_GBs']:.0f} GB/s algorithmic")

    n_acc, S_acc = args.c3_error_steps, args.c3_error_samples
    e_acc, h_acc = np.ascontiguousarray(eh[:, :S_acc]), np.ascontiguousarray(h[:, :S_acc])
    # the oracle on the first two sample columns, in worker processes while
    # the GPU runs below: its step size comes from its own element bound over
    # the whole ensemble (per element the largest E = (E h) / h)
    n_or = min(args.c3_oracle_steps, n_acc)
    oracle_pool = oracle_jobs = None
    if n_or > 0:
        ratio = np.concatenate([np.max(eh[i:i + 65536] / h[i:i + 65536], axis=1)
                                for i in range(0, eh.shape[0], 65536)])
        import multiprocessing as mp
        oracle_pool = mp.get_context("spawn").Pool(2)
        oracle_jobs = oracle_pool.map_async(_oracle_c3_column,
                                            [(np.ascontiguousarray(e_acc[:, s]), np.ascontiguousarray(h_acc[:, s]),
                                              ratio, n_or) for s in (0, 1)], chunksize=1)
        log(f"oracle started on sample columns 0 and 1, {n_or} steps")
    del eh, h
    ref_u = ref_q = None
    err = {}
    gpu_at = {}  # state and peak of columns 0, 1 after n_or steps, per mode
    for name, ap, st, _ in modes:
        ens = make(e_acc, h_acc, ap, st)
        ens.init_state()
        done = 0
        while done < n_acc:  # in chunks, with a progress line each
            k = min(10000, n_acc - done)
            if done < n_or:
                k = min(k, n_or - done)
            ens.step(k, dt, stream=stream)
            ens.sync()
            done += k
            log(f"  {name}: {done}/{n_acc} steps")
            if done == n_or:
                gpu_at[name] = (ens.read_state()[:, :2], ens.read_qoi()[:, :2])
        u, q = ens.read_state(), ens.read_qoi()
        ens.close()
        del ens
        torch.cuda.empty_cache()
        if ref_u is None:
            ref_u, ref_q = u, q
            continue
        err[name] = dict(state_rel_l2=float(np.linalg.norm(u - ref_u) / np.linalg.norm(ref_u)),
                         peak_rel_l2=float(np.linalg.norm(q - ref_q) / np.linalg.norm(ref_q)))
        log(f"{name}: after {n_acc} steps, state rel. L2 error {err[name]['state_rel_l2']:.2e}, "
            f"peak {err[name]['peak_rel_l2']:.2e} against FP64")
    vs_oracle = None
    if oracle_jobs is not None:
        waited = 0
        while not oracle_jobs.ready():  # progress lines while the oracle finishes
            oracle_jobs.wait(30)
            waited += 30
            log(f"  waiting for the oracle ({waited} s)")
        cols = oracle_jobs.get()
        oracle_pool.close()
        ou = np.stack([c[0] for c in cols], axis=1)
        oq = np.stack([c[1] for c in cols], axis=1)
        dt_or = cols[0][2]
        vs_oracle = {"steps": n_or, "samples": [0, 1], "dt_oracle_over_dt_gpu": dt_or / dt}
        for name, (gu, gq) in gpu_at.items():
            vs_oracle[name] = dict(
                state_rel_l2=float(np.linalg.norm(gu - ou) / np.linalg.norm(ou)),
                state_per_sample_max=float(np.max(np.linalg.norm(gu - ou, axis=0) / np.linalg.norm(ou, axis=0))),
                peak_rel_l2=float(np.linalg.norm(gq - oq) / np.linalg.norm(oq)))
            log(f"{name}: after {n_or} steps, state rel. L2 error {vs_oracle[name]['state_rel_l2']:.2e} "
                f"against the oracle (columns 0, 1)")
    head = thr["f32_apply_f64_state"]
    out = {
        "metric": "ensemble dof*sample*steps/s", "value": head["value"], "unit": "dof*sample*steps/s",
        "n_gpus": 1, "steps": steps, "warmup": 10, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 apply / f64 state", "data": "synthetic",
        "config": {"workload": "curved tapered tube 500x2000 nodes (3,000,000 dof), S=1,024 lognormal Matern E,h "
                               "(device-drawn), sine-ramped pulsatile pressure with axial taper and 1% shear, "
                               "alpha=50, dt=0.9 x element bound",
                   "n_dof": mesh.n_dof, "samples": S, "dt": dt, "parallelism": "single GPU"},
        "modes": thr,
        "error_vs_f64": {"steps": n_acc, "samples": S_acc, **err},
        "error_vs_oracle": vs_oracle,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1, help="must be 1: the benchmark runs on one GPU")
    ap.add_argument("--steps", type=int, default=2000, help="timed steps")
    ap.add_argument("--warmup", type=int, default=50, help="untimed steps before the timed ones")
    ap.add_argument("--apply", choices=["f32", "f64"], default="f32",
                    help="precision of the stiffness apply reported as value (state FP64)")
    ap.add_argument("--also-f64", action="store_true", default=True,
                    help="also time the other apply precision (default)")
    ap.add_argument("--no-also-f64", dest="also_f64", action="store_false",
                    help="skip timing the other apply precision")
    ap.add_argument("--no-cpu-baseline", dest="cpu", action="store_false", default=True,
                    help="skip timing the CPU oracle")
    ap.add_argument("--no-also-shared", dest="also_shared", action="store_false", default=True,
                    help="skip the shared-stiffness (block-row product) timing")
    ap.add_argument("--no-also-stress", dest="also_stress", action="store_false", default=True,
                    help="skip the wall-stress bands timing")
    ap.add_argument("--no-also-geom", dest="also_geom", action="store_false", default=True,
                    help="skip timing the geometry-refresh step")
    ap.add_argument("--geom-every", type=int, default=100, help="geometry refresh interval of that leg")
    ap.add_argument("--no-also-spde", dest="also_spde", action="store_false", default=True,
                    help="skip the SPDE field-sampler timing")
    ap.add_argument("--sample-block", type=int, default=0, help="0 = library default")
    ap.add_argument("--sb-inner", action="store_true", help="order workgroups sample-block fastest")
    ap.add_argument("--config", choices=["c2_cylinder", "c3_curved", "c4_batch", "c5_learned", "c5_kernels"],
                    default="c2_cylinder",
                    help="c2_cylinder: the headline single-mesh workload; c3_curved: the precision form at "
                         "1M nodes x 1,024 samples (about 6 GPU-minutes); c4_batch: the batching form; "
                         "c5_learned: the learned form (about 17 GPU-minutes); c5_kernels: the learned form's "
                         "kernels at full size on random data (training step, forward, moments)")
    ap.add_argument("--c3-error-steps", type=int, default=20000,
                    help="c3_curved: steps of the error run")
    ap.add_argument("--c3-error-samples", type=int, default=64,
                    help="c3_curved: sample columns of the error run (the first ones of the ensemble)")
    ap.add_argument("--c3-oracle-steps", type=int, default=2000,
                    help="c3_curved: steps of the oracle check on sample columns 0 and 1 (0: skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 10 times (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the ensemble shards over samples with no per-step "
              "exchange, and no multi-GPU figure is produced here (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.calib_copy:
        n = 1 << 30
        a = torch.empty(n // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": n, "calib_copy_bytes_written": n, "launches": 10}))
        return

    if args.config == "c3_curved":
        run_precision_config(args, torch)
        return
    if args.config == "c4_batch":
        run_batch_config(args, torch)
        return
    if args.config == "c5_learned":
        run_learned_config(args, torch)
        return
    if args.config == "c5_kernels":
        run_surrogate_kernels(args, torch)
        return

    from paper_2101_09059_amd import ensfem, inputs
    cfg = inputs.CONFIGS["c2_cylinder"]
    t0 = time.perf_counter()
    mesh = inputs.cylinder(cfg["R"], cfg["L"], cfg["n_theta"], cfg["n_z"])
    eh, h = inputs.lognormal_fields(mesh, cfg["S"], cfg["seed"])
    F = inputs.traction_load(mesh, cfg["p0"])
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s: {mesh.n_nodes} nodes, {mesh.n_el} tri, S={cfg['S']}")

    apply_ms = [None]

    def run(apply_f32: bool, steps: int, warmup: int, shared: bool = False, geom_every: int = 0):
        fields = np.repeat(eh[:, :1], eh.shape[1], axis=1) if shared else eh
        ens = ensfem.setup_case(mesh, fields, h, F, nu=cfg["nu"], shear_k=cfg["shear_k"], rho=cfg["rho"],
                                alpha=cfg["alpha"], apply_prec=ensfem.F32 if apply_f32 else ensfem.F64,
                                sample_block=args.sample_block, sb_inner=args.sb_inner, geom_every=geom_every)
        dt = ens.cfl_dt(cfg["safety"])
        ens.init_state()
        stream = torch.cuda.current_stream()
        ens.step(warmup, dt, stream=stream)
        ens.sync()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ens.step(steps, dt, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        ens.sync()
        info = ens.info()
        if apply_f32 and not shared and not geom_every:
            # stand-alone FP32 apply R = K(E h) U on [n_dof][S_pad] buffers
            dtype = torch.float32
            U = torch.randn(mesh.n_dof, info["S_pad"], device="cuda", dtype=dtype)
            R = torch.empty_like(U)
            n_app = 50
            for _ in range(5):
                ens.apply(U, R, ensfem.F32, stream=stream)
            e0.record(stream)
            for _ in range(n_app):
                ens.apply(U, R, ensfem.F32, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            apply_ms[0] = e0.elapsed_time(e1) / n_app
            del U, R
        ens.close()
        del ens
        torch.cuda.empty_cache()
        return ms, dt, info

    results = {}
    order = [args.apply == "f32"] + ([args.apply != "f32"] if args.also_f64 else [])
    for f32 in order:
        ms, dt, info = run(f32, args.steps, args.warmup)
        results["f32" if f32 else "f64"] = (ms, dt, info)
        log(f"apply={'f32' if f32 else 'f64'}: {ms / args.steps:.4f} ms/step")

    if args.also_shared:
        ms_sh, _, info_sh = run(args.apply == "f32", args.steps, args.warmup, shared=True)
        assert info_sh["variant"] == ensfem.VARIANT_CSR_SHARED
        log(f"shared stiffness, apply={args.apply}: {ms_sh / args.steps:.4f} ms/step")

    geom_out = None
    if args.also_geom:
        # geometry update: element matrices on each sample's moved geometry,
        # refreshed every --geom-every steps (the refresh copies included)
        ms_g, _, _ = run(args.apply == "f32", args.steps, args.warmup, geom_every=args.geom_every)
        geom_out = {"ms_per_step": ms_g / args.steps, "every": args.geom_every, "apply": args.apply}
        log(f"geometry refresh every {args.geom_every}, apply={args.apply}: {ms_g / args.steps:.4f} ms/step")

    stress_ms = None
    if args.also_stress:
        # wall-stress bands of the state after a short run (post-processing;
        # host-inclusive: the call synchronizes and returns per-element bands)
        ens = ensfem.setup_case(mesh, eh, h, F, nu=cfg["nu"], shear_k=cfg["shear_k"], rho=cfg["rho"],
                                alpha=cfg["alpha"], apply_prec=ensfem.F32, stress=True)
        ens.init_state()
        ens.step(200, ens.cfl_dt(cfg["safety"]))
        ens.sync()
        axial = np.tile([0.0, 0.0, 1.0], (mesh.n_el, 1))
        ens.stress_bands(axial, ensfem.STRESS_THETA_THETA)
        t0 = time.perf_counter()
        for comp in range(4):
            ens.stress_bands(axial, comp)
        stress_ms = (time.perf_counter() - t0) * 1e3 / 4
        ens.close()
        del ens
        torch.cuda.empty_cache()
        log(f"stress bands: {stress_ms:.1f} ms per component")

    spde_out = None
    if args.also_spde:
        # S Matern fields on the same mesh by the GPU SPDE sampler (kappa for
        # rho = 2 cm); host-inclusive (white noise in, fields out)
        sp = ensfem.Spde(mesh.xyz, mesh.tri, cfg["S"])
        z = np.random.default_rng(11).standard_normal((mesh.n_nodes, cfg["S"]))
        sp.sample(z[:, :], math.sqrt(2.0), tol=1e-8, max_iter=20000)
        t0 = time.perf_counter()
        _, it, res = sp.sample(z, math.sqrt(2.0), tol=1e-8, max_iter=20000)
        spde_ms = (time.perf_counter() - t0) * 1e3
        sp.close()
        del sp, z
        torch.cuda.empty_cache()
        spde_out = {"ms": spde_ms, "iterations": it, "relative_residual": res, "samples": cfg["S"],
                    "kappa": math.sqrt(2.0)}
        log(f"spde fields: {spde_ms:.0f} ms for {cfg['S']} samples, {it} CG iterations")

    ms, dt, info = results[args.apply]
    S = cfg["S"]
    work = mesh.n_dof * S * args.steps
    value = work / (ms * 1e-3)
    apply_f32 = args.apply == "f32"
    b = step_kernel_bytes(mesh.n_nodes, mesh.n_el, info["S_pad"], apply_f32)
    per_launch_s = ms * 1e-3 / args.steps
    achieved = b["total"] / per_launch_s / 1e9
    variant = f"fused_step_{args.apply}apply_f64state"
    traffic = measured_traffic("c2_cylinder", variant, b["total"])
    traffic, traffic_req = traffic if traffic else (None, None)
    out = {
        "metric": "ensemble dof*sample*steps/s",
        "value": value,
        "unit": "dof*sample*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 apply / f64 state" if apply_f32 else "f64",
        "data": "synthetic",
        "config": {"workload": "clamped cylinder 400x500 nodes (600,000 dof), S=256 lognormal Matern E,h, "
                               "steady pressure, alpha=50, dt=0.9 x element bound",
                   "n_dof": mesh.n_dof, "samples": S, "dt": dt, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"k_step ({variant})", "algorithmic_bytes_per_launch": b["total"],
                     "traffic_reads_by_request_size": traffic_req},
    }
    if apply_ms[0] is not None:
        # algorithmic bytes of the stand-alone apply: U read and R written
        # (4 B per dof and sample each), (E h) per element and sample, and the
        # per-mesh adjacency with its 3x6 blocks
        ab = (2 * mesh.n_dof * 4 + mesh.n_el * 4) * info["S_pad"] + 3 * mesh.n_el * (18 * 4 + 12)
        out["apply_only_f32"] = {"ms": apply_ms[0], "algorithmic_bytes": ab,
                                 "achieved_GBs": ab / (apply_ms[0] * 1e-3) / 1e9,
                                 "frac": ab / (apply_ms[0] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "kernel": "k_apply (node map: rows in the caller's numbering)"}
    if stress_ms is not None:
        out["stress_bands_ms_per_component"] = stress_ms
    if spde_out is not None:
        out["spde_fields"] = spde_out
    if geom_out is not None:
        out["geometry_refresh"] = geom_out
    if args.also_shared:
        out["ms_per_step_shared_stiffness"] = ms_sh / args.steps
        out["value_shared_stiffness"] = work / (ms_sh * 1e-3)
    for k, (ms2, _, _) in results.items():
        out[f"ms_per_step_{k}_apply"] = ms2 / args.steps
        out[f"value_{k}_apply"] = work / (ms2 * 1e-3)
    if args.cpu:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(mesh, eh, h, F, cfg, dt)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
