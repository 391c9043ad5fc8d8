"""Learned form: a surrogate of the per-node peak radial displacement used as
a multifidelity control variate for the plain ensemble solver.

Pipeline (every numerical step runs in the HIP library):
  1. inputs: the log-modulus and log-thickness fields are the truncated
     Karhunen-Loeve expansions of the nodal Matern field (Sec. 2.1) with
     n_modes coefficients each, so xi in R^(2 n_modes) determines a sample;
  2. data: the plain solver (FP32 apply / FP64 state) steps batches of
     samples under the pulsatile wall load and returns q = max_n e_r . u;
  3. training: the network xi -> standardized q (ensfem_surrogate.h) is
     fitted with Adam on the GPU, 90/10 train / held-out split;
  4. estimation: N fresh plain solves (high fidelity) and the network on the
     same xi, plus M further network draws reduced to per-node sums on the
     GPU, combined by the control-variate kernel; the estimate is used only
     if the median per-node correlation is >= 0.9 and the held-out relative
     RMSE is <= 5 %, otherwise the plain N-sample statistics are returned.

The host only draws xi, standardizes targets, orders batches and decides
the fallback.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import ensfem, inputs


class Problem:
    """One mesh, its KL basis and its load; solve(xi) -> peak radial q."""

    def __init__(self, mesh, cfg: dict, n_modes: int, sigma_log: float = 0.2, rho: float = 2.0):
        self.mesh, self.cfg, self.n_modes = mesh, cfg, n_modes
        self.lam, self.phi, self.captured = inputs.cylinder_kl_basis(mesh, n_modes, sigma_log, rho)
        self.F = inputs.traction_load(mesh, cfg["p0"])
        self.solve_seconds = 0.0
        self.solved = 0

    def fields(self, xi: np.ndarray):
        return inputs.kl_fields(self.mesh, self.lam, self.phi, xi[:, :self.n_modes], xi[:, self.n_modes:])

    def solve(self, xi: np.ndarray, return_moments: bool = False, progress=None):
        """Plain solver on the samples xi [S, 2 n_modes]; q [n_nodes, S].
        progress(str): optional callback told about each stage."""
        import torch
        c = self.cfg
        say = progress or (lambda m: None)
        t_a = time.perf_counter()
        eh, h = self.fields(xi)
        say(f"fields {time.perf_counter() - t_a:.1f} s")
        ens = ensfem.setup_case(self.mesh, eh, h, self.F, nu=c["nu"], shear_k=c["shear_k"], rho=c["rho"],
                                alpha=c["alpha"], kind=ensfem.LOAD_PULSATILE, t_ramp=c["T_ramp"],
                                amp=c["pulse_amp"], period=c["period"], apply_prec=ensfem.F32)
        del eh, h
        dt = ens.cfl_dt(c["safety"])
        steps = int(math.ceil(c["window"] / dt))
        say(f"set-up {time.perf_counter() - t_a:.1f} s, {steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.init_state()
        ens.step(steps, dt)
        ens.sync()
        self.solve_seconds += time.perf_counter() - t0
        self.solved += xi.shape[0]
        say(f"stepped {time.perf_counter() - t_a:.1f} s")
        q = ens.read_qoi()
        mom = ens.moments() if return_moments else None
        ens.close()
        return (q, mom) if return_moments else q


def draw_xi(seed: int, n: int, n_modes: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n, 2 * n_modes))


def he_normal_params(sizes, seed: int):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, FP32 vector."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(sizes[:-1], sizes[1:]):
        parts.append((rng.standard_normal((o, i), dtype=np.float32) * np.float32(math.sqrt(2.0 / i))).ravel())
        parts.append(np.zeros(o, np.float32))
    return np.concatenate(parts)


class Network:
    """The learned form's network plus target standardization."""

    def __init__(self, n_in: int, width: int, n_hidden: int, n_out: int, seed: int, max_batch: int = 256):
        self.net = ensfem.Surrogate(n_in, width, n_hidden, n_out, max_batch=max_batch)
        self.net.set_params(he_normal_params(self.net.sizes, seed))
        self.mu = np.zeros(n_out)
        self.sd = np.ones(n_out)
        self.max_batch = max_batch
        self.train_seconds = 0.0

    def fit(self, X: np.ndarray, Q: np.ndarray, epochs: int, batch: int, lr: float, seed: int,
            holdout: float = 0.1, val: float = 0.0, weight_decay: float = 0.0, eval_every: int = 10,
            progress=None):
        """X [N, n_in], Q [N, n_out] physical targets.  A `holdout` share is
        kept out for the reported relative RMSE; with `val` > 0 a further
        share is used for early stopping (the parameters with the lowest
        validation RMSE, checked every `eval_every` epochs, are kept).
        Returns the held-out relative RMSE (physical units) and the loss
        history (last batch loss of each epoch).  progress(str): optional
        callback told about each validation check."""
        import torch
        rng = np.random.default_rng(seed)
        N = X.shape[0]
        perm = rng.permutation(N)
        n_hold = max(1, int(round(holdout * N)))
        n_val = int(round(val * N))
        hold, vset, train = perm[:n_hold], perm[n_hold:n_hold + n_val], perm[n_hold + n_val:]
        Qtr = Q[train]
        self.mu = Qtr.mean(axis=0)
        sd = Qtr.std(axis=0)
        # outputs that never vary (clamped nodes) are predicted by their mean
        self.sd = np.where(sd > 0, sd, 0.0)
        scale = np.where(sd > 0, sd, 1.0)
        self.net.set_weight_decay(weight_decay)
        dev = "cuda"
        Xt = torch.as_tensor(X[train], dtype=torch.float32, device=dev)
        Tt = torch.as_tensor((Qtr - self.mu) / scale, dtype=torch.float32, device=dev)
        del Qtr
        n_tr = Xt.shape[0]
        # validation set on the device: its error and the best parameters
        # stay there between checks
        if n_val:
            Xv = torch.as_tensor(X[vset], dtype=torch.float32, device=dev)
            Qv = torch.as_tensor(Q[vset], dtype=torch.float64, device=dev)
            qv_norm = float(np.linalg.norm(Q[vset]))
            mu_t = torch.as_tensor(self.mu, dtype=torch.float64, device=dev)
            sd_t = torch.as_tensor(self.sd, dtype=torch.float64, device=dev)
            sq_t = torch.zeros(1, dtype=torch.float64, device=dev)
            best_dev = torch.empty(self.net.n_params, dtype=torch.float32, device=dev)
        xb = torch.empty((batch, Xt.shape[1]), dtype=torch.float32, device=dev)
        tb = torch.empty((batch, Tt.shape[1]), dtype=torch.float32, device=dev)
        steps_per_epoch = int(math.ceil(n_tr / batch))
        total = epochs * steps_per_epoch
        hist = []
        best = (np.inf, None, 0)
        self.val_history = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step = 0
        for ep in range(epochs):
            order = torch.as_tensor(rng.permutation(n_tr).astype(np.int32), device=dev)
            for b0 in range(0, n_tr, batch):
                idx = order[b0:b0 + batch]
                xs = self.net.gather_rows(Xt, idx, xb)
                ts = self.net.gather_rows(Tt, idx, tb)
                lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * step / total))
                loss = self.net.train_step(xs, ts, lr_t)
                step += 1
            hist.append(float(loss.item()))
            if n_val and ((ep + 1) % eval_every == 0 or ep + 1 == epochs):
                sq_t.zero_()
                for r0 in range(0, Xv.shape[0], self.max_batch):
                    self.net.sq_error(Xv[r0:r0 + self.max_batch], Qv[r0:r0 + self.max_batch], mu_t, sd_t, sq_t)
                e = math.sqrt(float(sq_t.item())) / qv_norm
                self.val_history.append((ep + 1, e))
                if e < best[0]:
                    self.net.get_params_device(best_dev)
                    best = (e, best_dev, ep + 1)
                if progress:
                    progress(f"  epoch {ep + 1}/{epochs}: loss {hist[-1]:.3e}, validation rel RMSE {e:.4f}")
        if best[1] is not None:
            self.net.set_params(best[1].cpu().numpy())
        self.best_epoch = best[2] if best[1] is not None else epochs
        torch.cuda.synchronize()
        self.train_seconds += time.perf_counter() - t0
        pred = self.predict(X[hold])
        rmse = float(np.linalg.norm(pred - Q[hold]) / np.linalg.norm(Q[hold]))
        return rmse, hist

    def predict(self, X: np.ndarray) -> np.ndarray:
        """Physical-unit predictions [rows, n_out] (host)."""
        import torch
        out = []
        Xt = torch.as_tensor(X, dtype=torch.float32, device="cuda")
        for r0 in range(0, X.shape[0], self.max_batch):
            out.append(self.net.forward(Xt[r0:r0 + self.max_batch]).cpu().numpy().astype(np.float64))
        Y = np.concatenate(out)
        return self.mu + self.sd * Y

    def moment_sums(self, X: np.ndarray):
        """Sums of q and q^2 per output over the rows of X, physical units;
        the rows' outputs are reduced on the GPU and never stored."""
        import torch
        M = X.shape[0]
        s1, s2 = self.net.moments(torch.as_tensor(X, dtype=torch.float32, device="cuda"))
        mu, sd = self.mu, self.sd
        return M * mu + sd * s1, M * mu * mu + 2.0 * mu * sd * s1 + sd * sd * s2

    def close(self):
        self.net.close()


def estimate(qH: np.ndarray, plain_mean: np.ndarray, plain_var: np.ndarray, qL: np.ndarray,
             sumL: np.ndarray, sumsqL: np.ndarray, M: int, heldout_rmse: float,
             rho_min: float = 0.9, rmse_max: float = 0.05):
    """Control-variate statistics with the fallback rule.  plain_mean /
    plain_var are the high-fidelity ensemble's own statistics, returned
    unchanged when the surrogate does not qualify."""
    mean, var, rho = ensfem.cv_moments(qH, qL, sumL, sumsqL, M)
    active = qH.var(axis=1) > 0
    rho_med = float(np.median(rho[active])) if active.any() else 0.0
    use = rho_med >= rho_min and heldout_rmse <= rmse_max
    if not use:
        return dict(mean=plain_mean, var=plain_var, rho=rho, rho_median=rho_med, used_cv=False)
    return dict(mean=mean, var=var, rho=rho, rho_median=rho_med, used_cv=True)


def bootstrap_variance_ratio(qH: np.ndarray, qL: np.ndarray, sumL: np.ndarray, M: int, n_boot: int = 200,
                             n_nodes: int = 4096, seed: int = 0) -> float:
    """Variance-reduction factor of the control-variate mean measured by
    resampling the N high-fidelity pairs (diagnostic, host side): for each
    bootstrap replicate the plain mean and the control-variate mean (with
    its own beta) are formed on a random subset of varying nodes; returns the
    median over nodes of var(plain) / var(CV) across replicates."""
    rng = np.random.default_rng(seed)
    act = np.flatnonzero(qH.var(axis=1) > 0)
    nodes = rng.choice(act, size=min(n_nodes, act.size), replace=False)
    H, L = qH[nodes], qL[nodes]
    muL = sumL[nodes] / M
    N = H.shape[1]
    plain = np.empty((n_boot, nodes.size))
    cv = np.empty((n_boot, nodes.size))
    for b in range(n_boot):
        idx = rng.integers(0, N, N)
        h, l = H[:, idx], L[:, idx]
        mh, ml = h.mean(1), l.mean(1)
        cov = ((h - mh[:, None]) * (l - ml[:, None])).sum(1) / (N - 1)
        var = l.var(1, ddof=1)
        beta = np.where(var > 0, cov / np.where(var > 0, var, 1.0), 0.0)
        plain[b] = mh
        cv[b] = mh - beta * (ml - muL)
    vp, vc = plain.var(0), cv.var(0)
    ok = vc > 0
    return float(np.median(vp[ok] / vc[ok])) if ok.any() else float("nan")
