"""Subspace-size estimator on the device: the perceptron's forward pass, gradients and Adam step
against the FP64 reference network, the stochastic trace features against the closed-form trace
of the filter, the rank check, and the estimator end to end on held-out pencils."""
import numpy as np
import pytest

import pencils
from oracle import brute, mlp
from oracle import quadrature as Q
from tests.gpu_common import device, match_eigs

pytestmark = pytest.mark.gpu


def fm():
    import paper_1404_2891_amd as m
    return m


def torch():
    import torch as t
    return t


def f32(a):
    return torch().from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device())


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / np.linalg.norm(b))


def problem(seed=0, batch=200, n_in=19, hidden=256):
    g = np.random.default_rng(seed)
    P = mlp.init_params(g, n_in, hidden)
    X = g.standard_normal((batch, n_in)) * 2.0 + 0.5
    t = g.uniform(0, 48, size=batch)
    return P, X, t


@pytest.mark.parametrize("half,tol", [(False, 1e-5), (True, 2e-2)])
def test_gradients_match_reference(half, tol):
    P, X, t = problem(1)
    net = fm().MLP(mlp.flatten(P), half=half, max_batch=256, device=device())
    g, loss = net.gradients(f32(X), f32(t))
    y, cache = mlp.forward(P, X)
    gref = mlp.flatten(mlp.backward(P, cache, y, t))
    assert rel(g.cpu().numpy(), gref) < tol
    assert abs(loss - mlp.mse(y, t)) < 10 * tol * mlp.mse(y, t)
    net.close()


@pytest.mark.parametrize("half,tol", [(False, 1e-6), (True, 5e-3)])
def test_forward_with_standardization(half, tol):
    """Inputs standardised with the measured column moments (population variance)."""
    P, X, t = problem(2, batch=300)
    net = fm().MLP(mlp.flatten(P), half=half, max_batch=512, device=device())
    Xd = f32(X)
    net.fit_standardization(Xd)
    y = net.forward(Xd).cpu().numpy()
    Xs = (X.astype(np.float32).astype(np.float64) - X.astype(np.float32).mean(axis=0)) / X.astype(np.float32).std(axis=0)
    yref, _ = mlp.forward(P, Xs)
    assert rel(y, yref) < tol
    net.close()


def test_adam_step_matches_reference():
    """One FP32 training step moves the parameters as the reference Adam step does (the first step
    moves each by about -lr sign(g)); entries whose gradient is near zero may differ in sign."""
    P, X, t = problem(3)
    net = fm().MLP(mlp.flatten(P), half=False, max_batch=256, device=device())
    net.train_step(f32(X), f32(t), lr=1e-3)
    got = net.params().astype(np.float64) - mlp.flatten(P).astype(np.float32)
    y, cache = mlp.forward(P, X)
    P1 = mlp.adam_step({k: v.copy() for k, v in P.items()}, mlp.backward(P, cache, y, t), mlp.adam_init(P), 1, lr=1e-3)
    want = mlp.flatten(P1) - mlp.flatten(P)
    bad = np.abs(got - want) > 1e-5
    assert bad.mean() < 5e-3, bad.mean()
    net.close()


def test_training_reduces_loss():
    g = np.random.default_rng(4)
    X = g.uniform(-1, 1, size=(2048, 19))
    t = 20 + 10 * np.sin(2 * X[:, 0]) + 5 * X[:, 1] * X[:, 2]
    P = mlp.init_params(g)
    net = fm().MLP(mlp.flatten(P), half=True, max_batch=256, device=device())
    Xd, td = f32(X), f32(t)
    net.fit_standardization(Xd)
    first = None
    for epoch in range(40):
        for b in range(0, 2048, 256):
            loss = net.train_step(Xd[b:b + 256], td[b:b + 256], lr=2e-3, want_loss=(b == 0))
            if first is None:
                first = loss
    y = net.forward(Xd[:256]).cpu().numpy()
    assert np.mean((y - t[:256]) ** 2) < 0.02 * first
    net.close()


def probe_batch(P, V, precision="fp32"):
    """Probe contexts (8 trapezoid nodes, no refinement) of a list of pencils.  FP32 factorisations:
    with FP16 updates the solve error of these node systems (kappa u16 of order one) exceeds the
    estimator's own noise."""
    dev = [(fm().to_device(p.A, device()) if isinstance(p.A, np.ndarray) else p.A, None) for p in P]
    contours = [(p.center, p.radius, 1.0) for p in P]
    b = fm().FeastBatch(dev, contours, m0=8, q=8, precision=precision, ir_max=0)
    feats = np.array([b.member_probe_features(i, V) for i in range(len(P))])
    b.close()
    return feats


def test_probe_features_estimate_the_filter_trace():
    """mean_j v_j^H rho_8(M) v_j estimates trace rho_8(M) = sum_i rho_8(lambda_i) (closed form of the
    8-node trapezoid filter); with Rademacher probes its variance is the off-diagonal squared
    Frobenius norm of rho_8(M) over the probe count, so the mean lies within 5 standard errors."""
    n = 512
    V = fm().to_device(pencils.probe_block(4, 0, n), device())
    ids = pencils.c4_split("train", 6)
    P = [pencils.c4_pencil(j, n, basis=b) for j, b in ids]
    feats = probe_batch(P, V)
    for (j, b), p, f in zip(ids, P, feats):
        mu = (p.lam - p.center) / p.radius
        rho = 1.0 / (1.0 - mu ** 8)
        trace = rho.sum()
        U, s, W = pencils.c4_basis(b, n)
        Vb = (U * s) @ W.conj().T
        Rm = (Vb * rho) @ np.linalg.inv(Vb)
        off = np.linalg.norm(Rm) ** 2 - np.sum(np.abs(np.diag(Rm)) ** 2)
        se = np.sqrt(off / 8)
        est = complex(f[0:16:2].mean(), f[1:16:2].mean())
        assert abs(est - trace) < 5 * se + 0.05 * abs(trace) + 0.5, (est, trace, se)
        assert np.allclose(f[16:], [p.center.real, p.center.imag, p.radius], rtol=1e-6)


def test_rank_check_flags_a_small_subspace():
    """m0 = 8 < m = 10 (C0 pencil): no gap in the filtered block's singular values and every Ritz
    value inside, so the run stops after one iteration with FEAST_ERANK; m0 = 16 passes the check
    (about 10 Ritz values inside) and converges."""
    P = pencils.c0()
    A = fm().to_device(P.A, device())
    small = fm().Feast(A, None, 0j, 1.0, 1.0, 16, 8, rank_check=True)
    r = small.iterate(fm().to_device(pencils.start_block(0, P.n, 8), device()))
    assert r.code == fm().binding.FEAST_ERANK and r.iterations == 1 and r.rank == 8
    small.close()
    ok = fm().Feast(A, None, 0j, 1.0, 1.0, 16, 16, rank_check=True)
    r = ok.iterate(fm().to_device(pencils.start_block(0, P.n, 16), device()))
    assert r.code == 0 and r.converged and len(r.lam) == 10
    assert 10 <= r.rank <= 16
    ok.close()


def test_estimator_end_to_end_on_held_out_pencils():
    """Features of 768 training pencils (probes with FP32 factorisations), labels = the prescribed
    counts, 120 epochs of Adam.  On 48 held-out pencils (other seeds, other bases) the estimate
    beats the constant predictor (the features carry the count through their noise), and the
    pipeline m0 = rule(estimate), FEAST with the rank check, m0 doubled on FEAST_ERANK, finds every
    pencil's eigenvalues inside its contour."""
    n, ntr, nev = 512, 768, 48
    dev = device()
    V = fm().to_device(pencils.probe_block(4, 0, n), dev)
    tr = [pencils.c4_pencil(j, n, basis=b, device=dev) for j, b in pencils.c4_split("train", ntr)]
    ev = [pencils.c4_pencil(j, n, basis=b, device=dev) for j, b in pencils.c4_split("eval", nev)]
    Xtr = np.concatenate([probe_batch(tr[i:i + 64], V) for i in range(0, ntr, 64)])
    Xev = probe_batch(ev, V)
    ytr = np.array([p.m for p in tr], dtype=np.float32)
    yev = np.array([p.m for p in ev], dtype=np.float64)
    net = fm().MLP(mlp.flatten(mlp.init_params(np.random.default_rng(7))), half=True, max_batch=256, device=dev)
    Xd, yd = f32(Xtr), f32(ytr)
    net.fit_standardization(Xd)
    order = np.random.default_rng(8)
    losses = []
    for epoch in range(120):
        perm = torch().from_numpy(order.permutation(ntr)).to(dev)
        Xp, yp = Xd[perm].contiguous(), yd[perm].contiguous()
        for b in range(0, ntr, 128):
            loss = net.train_step(Xp[b:b + 128], yp[b:b + 128], lr=1e-3, want_loss=(b == 0))
            if b == 0:
                losses.append(loss)
    assert np.mean(losses[-10:]) < 0.5 * losses[0]
    m_hat = net.forward(f32(Xev)).cpu().numpy().astype(np.float64)
    mse_net = np.mean((m_hat - yev) ** 2)
    mse_const = np.mean((ytr.mean() - yev) ** 2)
    assert mse_net < mse_const, (mse_net, mse_const)
    for p, mh in zip(ev, m_hat):
        m0 = fm().m0_from_estimate(mh)
        while True:
            F = fm().Feast(p.A, None, p.center, p.radius, 1.0, 16, m0, rank_check=True)
            r = F.iterate(fm().to_device(pencils.start_block(4, n, m0), dev))
            F.close()
            if r.code != fm().binding.FEAST_ERANK or m0 >= n:
                break
            m0 = min(2 * m0, n)
        assert r.converged and len(r.lam) == p.m, (p.name, mh, m0, len(r.lam), p.m)
        assert match_eigs(r.lam, brute.eigenvalues_inside(p.lam, p.center, p.radius)) < 1e-9
    net.close()


@pytest.mark.parametrize("half", [False, True])
def test_estimate_m0_chains_probes_network_and_rule(half):
    """feast_estimate_m0 in one call = feast_probe_features, the perceptron's forward pass on those
    features and feast_m0_from_estimate (capped at n), each also called separately here; a
    perceptron of the wrong input width is rejected."""
    n = 512
    dev = device()
    V = fm().to_device(pencils.probe_block(4, 0, n), dev)
    g = np.random.default_rng(12)
    P0 = mlp.init_params(g, 19, 64)
    # scale the last layer so that estimates land in the range of real counts
    P0["W3"] = P0["W3"] * 20.0
    P0["b3"] = P0["b3"] + 24.0
    net = fm().MLP(mlp.flatten(P0), n_in=19, hidden=64, half=half, max_batch=8, device=dev)
    for j, b in pencils.c4_split("eval", 3):
        p = pencils.c4_pencil(j, n, basis=b)
        with fm().Feast(fm().to_device(p.A, dev), None, p.center, p.radius, 1.0, 8, 8, precision="fp32",
                        ir_max=0) as F:
            m0, m_hat = F.estimate_m0(net, V)
            feats = F.probe_features(V)
        want = float(net.forward(f32(feats[None, :])).cpu().numpy()[0])
        y_ref, _ = mlp.forward(P0, feats[None, :].astype(np.float64))
        assert abs(m_hat - want) <= 1e-5 * max(1.0, abs(want)), (m_hat, want)
        assert abs(m_hat - y_ref[0]) <= (5e-3 if half else 1e-5) * max(1.0, abs(y_ref[0]))
        assert m0 == min(n, fm().m0_from_estimate(m_hat))
    bad = fm().MLP(mlp.flatten(mlp.init_params(g, 11, 16)), n_in=11, hidden=16, half=half, max_batch=4, device=dev)
    p = pencils.c4_pencil(0, n, basis=0)
    with fm().Feast(fm().to_device(p.A, dev), None, p.center, p.radius, 1.0, 8, 8, precision="fp32", ir_max=0) as F:
        with pytest.raises(fm().FeastError) as e:
            F.estimate_m0(bad, V)
        assert e.value.code == -5
    net.close()
    bad.close()
