"""Learned form on the GPU: BF16-MFMA network kernels against the FP64
oracle network (at BF16-rounded weights and inputs), one Adam step, the
moments-over-draws epilogue, and the control-variate kernel.

Tolerances: BF16 activations between layers give ~4e-3 relative rounding
per layer, so outputs and gradients are compared at 2e-2 / 3e-2 relative;
FP32 and FP64 reductions at 1e-5 and 1e-12."""
import numpy as np
import pytest

from oracle import control_variate as ocv
from oracle import mlp
from paper_2101_09059_amd import ensfem
from tests._cases import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def bf16_round(x):
    """Round-to-nearest-even to BF16, returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _net(sizes, seed, bias_scale=0.1):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(sizes, rng)
    p = [(bf16_round(W), rng.standard_normal(b.shape) * bias_scale) for W, b in p]
    return p


@pytest.mark.parametrize("sizes,batch", [([20, 72, 72, 150], 37), ([128, 256, 256, 256, 1000], 256),
                                         ([16, 64, 130], 129)])
def test_forward_matches_oracle(sizes, batch):
    say(f"case: surrogate forward sizes={sizes} batch={batch}")
    params = _net(sizes, seed=len(sizes) + batch)
    rng = np.random.default_rng(1)
    X = bf16_round(rng.standard_normal((batch, sizes[0])))
    net = ensfem.Surrogate(sizes[0], sizes[1], len(sizes) - 2, sizes[-1], max_batch=max(batch, 64))
    net.set_params(ensfem.flatten_params(params))
    Y = net.forward(torch.as_tensor(X, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    ref, _ = mlp.forward([(W, b.astype(np.float32).astype(np.float64)) for W, b in params], X)
    err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    say(f"  rel err {err:.2e}")
    assert err < 2e-2
    net.close()


@pytest.mark.parametrize("sizes,batch", [([24, 64, 64, 40], 48), ([128, 128, 128, 520], 64)])
def test_gradients_match_oracle(sizes, batch):
    say(f"case: surrogate gradients sizes={sizes}")
    params = _net(sizes, seed=7)
    rng = np.random.default_rng(2)
    X = bf16_round(rng.standard_normal((batch, sizes[0])))
    T = rng.standard_normal((batch, sizes[-1]))
    net = ensfem.Surrogate(sizes[0], sizes[1], len(sizes) - 2, sizes[-1], max_batch=batch)
    net.set_params(ensfem.flatten_params(params))
    g, loss = net.gradients(torch.as_tensor(X, dtype=torch.float32, device="cuda"),
                            torch.as_tensor(T, dtype=torch.float32, device="cuda"))
    g = g.double().cpu().numpy()
    p64 = [(W, b.astype(np.float32).astype(np.float64)) for W, b in params]
    Y, cache = mlp.forward(p64, X)
    ref = ensfem.flatten_params(mlp.backward(p64, cache, Y, T)).astype(np.float64)
    gl = ensfem.unflatten_params(g, sizes)
    rl = ensfem.unflatten_params(ref, sizes)
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(gl, rl)):
        eW = np.linalg.norm(gW - rW) / np.linalg.norm(rW)
        eb = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
        say(f"  layer {li}: dW {eW:.2e}  db {eb:.2e}")
        assert eW < 3e-2 and eb < 3e-2
    assert abs(float(loss.item()) / mlp.loss(Y, T) - 1) < 1e-2
    net.close()


@pytest.mark.parametrize("wd", [0.0, 0.3])
def test_adam_step_matches_oracle(wd):
    sizes, batch = [32, 64, 64, 48], 32
    params = _net(sizes, seed=11)
    rng = np.random.default_rng(3)
    X = bf16_round(rng.standard_normal((batch, sizes[0])))
    T = rng.standard_normal((batch, sizes[-1]))
    net = ensfem.Surrogate(sizes[0], sizes[1], 2, sizes[-1], max_batch=batch)
    p0 = ensfem.flatten_params(params)
    net.set_params(p0)
    net.set_weight_decay(wd)
    lr = 1e-3
    Xt = torch.as_tensor(X, dtype=torch.float32, device="cuda")
    Tt = torch.as_tensor(T, dtype=torch.float32, device="cuda")
    g_gpu = net.gradients(Xt, Tt)[0].double().cpu().numpy()
    net.train_step(Xt, Tt, lr)
    p1 = net.get_params().astype(np.float64)
    # the update must be Adam's first step on the GPU's own gradient
    gl = ensfem.unflatten_params(g_gpu, sizes)
    zeros = [(np.zeros_like(W), np.zeros_like(b)) for W, b in gl]
    p0l = ensfem.unflatten_params(p0.astype(np.float64), sizes)
    newp, _, _ = mlp.adam_step(p0l, gl, zeros, zeros, 1, lr, weight_decay=wd)
    ref = ensfem.flatten_params(newp).astype(np.float64)
    assert np.max(np.abs(p1 - ref)) <= 1e-6
    # and follow the FP64 oracle's step direction on almost every entry
    Y, cache = mlp.forward([(W, b.astype(np.float32).astype(np.float64)) for W, b in params], X)
    r = ensfem.flatten_params(mlp.backward(params, cache, Y, T)).astype(np.float64)
    big = np.abs(r) > 1e-2 * np.abs(r).max()
    assert np.mean(np.sign(g_gpu[big]) == np.sign(r[big])) > 0.98
    net.close()


def test_moments_match_explicit_forward():
    sizes = [128, 128, 128, 777]
    params = _net(sizes, seed=5)
    rng = np.random.default_rng(4)
    M = 1000
    X = torch.as_tensor(rng.standard_normal((M, sizes[0])), dtype=torch.float32, device="cuda")
    net = ensfem.Surrogate(sizes[0], sizes[1], 2, sizes[-1], max_batch=256)
    net.set_params(ensfem.flatten_params(params))
    s1, s2 = net.moments(X)
    Y = torch.cat([net.forward(X[i:i + 256]) for i in range(0, M, 256)]).double().cpu().numpy()
    assert np.allclose(s1, Y.sum(0), rtol=1e-5, atol=1e-5 * np.abs(Y).sum(0).max())
    assert np.allclose(s2, (Y * Y).sum(0), rtol=1e-5)
    net.close()


@pytest.mark.parametrize("sizes,M", [([24, 72, 72, 150], 5000), ([128, 256, 256, 256, 1000], 4500),
                                     ([16, 60, 130], 300)])
def test_moments_match_oracle(sizes, M):
    """sur_moments (hidden layers per pass of 4,096 rows, the output layer
    through the first and second moments of the last hidden layer) against
    the oracle's explicit forward of every row, summed in FP64: two passes
    with a ragged tail, ragged tiles, a width that is not a multiple of 8."""
    say(f"case: surrogate moments sizes={sizes} M={M}")
    params = _net(sizes, seed=len(sizes) + M)
    rng = np.random.default_rng(12)
    X = bf16_round(rng.standard_normal((M, sizes[0])))
    net = ensfem.Surrogate(sizes[0], sizes[1], len(sizes) - 2, sizes[-1], max_batch=64)
    net.set_params(ensfem.flatten_params(params))
    s1, s2 = net.moments(torch.as_tensor(X, dtype=torch.float32, device="cuda"))
    Y, _ = mlp.forward([(W, b.astype(np.float32).astype(np.float64)) for W, b in params], X)
    r1, r2, a1 = Y.sum(0), (Y * Y).sum(0), np.abs(Y).sum(0)
    e1 = np.linalg.norm(s1 - r1) / np.linalg.norm(a1)
    e2 = np.linalg.norm(s2 - r2) / np.linalg.norm(r2)
    say(f"  sum y: err {e1:.2e} of the sum of |y|; sum y^2: rel err {e2:.2e}")
    assert e1 < 2e-2 and e2 < 4e-2
    net.close()


def test_training_reduces_loss():
    sizes, batch = [16, 128, 128, 64], 128
    rng = np.random.default_rng(6)
    params = mlp.init_params(sizes, rng)
    X = rng.standard_normal((batch, 16))
    A = rng.standard_normal((16, 64)) / 4
    T = np.tanh(X @ A) + 0.1 * (X[:, :1] ** 2)
    net = ensfem.Surrogate(16, 128, 2, 64, max_batch=batch)
    net.set_params(ensfem.flatten_params(params))
    Xt = torch.as_tensor(X, dtype=torch.float32, device="cuda")
    Tt = torch.as_tensor(T, dtype=torch.float32, device="cuda")
    first = float(net.train_step(Xt, Tt, 1e-3).item())
    for _ in range(300):
        net.train_step(Xt, Tt, 1e-3)
    last = float(net.train_step(Xt, Tt, 1e-3).item())
    say(f"  loss {first:.3e} -> {last:.3e}")
    assert last < 0.1 * first
    net.close()


def test_control_variate_kernel_matches_oracle():
    rng = np.random.default_rng(8)
    n, N, M = 333, 64, 5000
    qH = rng.standard_normal((n, N)) * 0.3 + 2
    qL = qH + 0.05 * rng.standard_normal((n, N))
    Lp = 2 + 0.3 * rng.standard_normal((n, M))
    s1, s2 = Lp.sum(1), (Lp * Lp).sum(1)
    mean, var, rho = ensfem.cv_moments(qH, qL, s1, s2, M)
    ref = ocv.cv_moments(qH, qL, s1, s2, M)
    assert np.allclose(mean, ref["mean"], rtol=1e-12, atol=0)
    assert np.allclose(var, ref["var"], rtol=1e-10, atol=1e-14)
    assert np.allclose(rho, ref["rho"], rtol=1e-12, atol=0)


def test_squared_error_and_row_gather():
    """sur_sq_error: the physical-unit squared error of the network's own
    forward output, accumulated over two batches, against numpy in FP64 on
    that output (1e-12); sur_gather_rows: rows copied exactly."""
    sizes, rows = [16, 64, 64, 300], 70
    say("case: surrogate squared error and row gather")
    params = _net(sizes, seed=3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((rows, sizes[0]))
    net = ensfem.Surrogate(sizes[0], sizes[1], len(sizes) - 2, sizes[-1], max_batch=40)
    net.set_params(ensfem.flatten_params(params))
    Xd = torch.as_tensor(X, dtype=torch.float32, device="cuda")
    mu = rng.standard_normal(sizes[-1])
    sd = np.abs(rng.standard_normal(sizes[-1]))
    sd[::7] = 0.0
    Q = rng.standard_normal((rows, sizes[-1]))
    mu_d, sd_d = torch.as_tensor(mu, device="cuda"), torch.as_tensor(sd, device="cuda")
    Q_d = torch.as_tensor(Q, device="cuda")
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    ref = 0.0
    for r0 in (0, 40):
        net.sq_error(Xd[r0:r0 + 40], Q_d[r0:r0 + 40], mu_d, sd_d, acc)
        y = net.forward(Xd[r0:r0 + 40]).cpu().numpy().astype(np.float64)
        ref += float(np.sum((mu + sd * y - Q[r0:r0 + 40]) ** 2))
    torch.cuda.synchronize()
    assert abs(float(acc.item()) - ref) <= 1e-12 * ref
    idx = torch.as_tensor(rng.permutation(rows)[:33].astype(np.int32), device="cuda")
    out = torch.full((40, sizes[0]), float("nan"), dtype=torch.float32, device="cuda")
    got = net.gather_rows(Xd, idx, out)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), Xd.cpu().numpy()[idx.cpu().numpy()])
    net.close()
