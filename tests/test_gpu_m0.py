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


def test_estimator_gains_over_the_method_without_it():
    """The learned part end to end.  Training: 1,536 pencils labelled by the count the plain FP64
    FEAST run finds (q = 16, m0 = 64), with the probe features of that run's own filter; 80 epochs
    of Adam on the perceptron (FP16 operands).  Held out: 256 pencils (other seeds, other bases)
    solved in FP32 with the rank check and restarts on the same factorisations, m0 from (a) the
    estimator, (b) a fixed 64 (enough for every count here: no restarts), (c) 1.5 x the mean probe
    trace (the features without the network).  Every strategy finds every pencil's eigenvalues
    inside its contour; the estimator's algorithmic work (factorisations + probe solves +
    iterations, restarts included) is below both others'."""
    n, ntr, nev = 512, 1536, 256
    dev = device()
    V = fm().to_device(pencils.probe_block(4, 0, n), dev)
    X, y = [], []
    ids = pencils.c4_split("train", ntr)
    for i0 in range(0, ntr, 512):
        part = [pencils.c4_pencil(j, n, basis=b, device=dev) for j, b in ids[i0:i0 + 512]]
        b = fm().FeastBatch([(p.A, None) for p in part], [(p.center, p.radius, 1.0) for p in part], m0=64, q=16,
                            precision="fp64")
        X += list(b.probe_features(V))
        res, rcs = b.iterate([fm().to_device(pencils.start_block(4, n, 64), dev) for _ in part])
        b.close()
        labels = [len(r.lam) for r in res]
        assert labels == [p.m for p in part]   # the method's counts are the constructed ones
        y += labels
    X, y = np.array(X), np.array(y, dtype=np.float32)
    net = fm().MLP(mlp.flatten(mlp.init_params(np.random.default_rng(7), X.shape[1])), n_in=X.shape[1], half=True,
                   max_batch=512, device=dev)
    Xd, yd = f32(X), f32(y)
    net.fit_standardization(Xd)
    order = np.random.default_rng(8)
    for epoch in range(80):
        perm = torch().from_numpy(order.permutation(ntr)).to(dev)
        Xp, yp = Xd[perm].contiguous(), yd[perm].contiguous()
        for b in range(0, ntr, 128):
            net.train_step(Xp[b:b + 128], yp[b:b + 128], lr=1e-3)
    ev = [pencils.c4_pencil(j, n, basis=b, device=dev) for j, b in pencils.c4_split("eval", nev)]

    def estimator(feats, i0):
        m_hat = net.forward(f32(feats)).cpu().numpy().astype(np.float64)
        return [fm().m0_from_estimate(v) for v in m_hat]

    def probe_mean(feats, i0):
        t = feats[:, 0:2 * V.shape[1]:2].mean(axis=1)
        return [max(8, int(np.ceil(1.5 * max(x, 0.0) / 8.0)) * 8) for x in t]

    work = {}
    for name, rule, cap in (("estimator", estimator, 128), ("fixed_64", None, 64), ("probe_mean", probe_mean, 128)):
        res, m0s, restarts, w = fm().binding.sized_solve(
            [(p.A, None) for p in ev], [(p.center, p.radius, 1.0) for p in ev],
            lambda i, m0: fm().to_device(pencils.start_block(4, n, m0), dev), m0_rule=rule, cap=cap, probes=V)
        for p, r in zip(ev, res):
            ref = brute.eigenvalues_inside(p.lam, p.center, p.radius)
            assert r.converged and len(r.lam) == p.m == len(ref), (name, p.name, len(r.lam), p.m)
            if p.m:
                assert match_eigs(r.lam, ref) < 1e-9
        work[name] = sum(w.values())
        print(name, f"{work[name] / nev / 1e9:.2f} GFLOP per pencil, mean m0 {np.mean(m0s):.1f}, {restarts} restarts")
    assert work["estimator"] < 0.95 * work["fixed_64"], work
    assert work["estimator"] < 0.98 * work["probe_mean"], work
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


@pytest.mark.parametrize("mode", ["grouped", "streams"])
def test_empty_contours_terminate_in_fp32(mode):
    """Held-out pencils 105 and 109 of the learned-m0 set have no eigenvalue inside their circle
    (m = 0); with m0 = 64 the FP32 iteration's Ritz values of the filtered noise kept landing inside
    and the empty-set rule (no Ritz value inside twice in a row) never held in 30 iterations.  The
    filter-gain rule ends them with m = 0, and the pencils around them keep their counts."""
    ids = [104, 105, 106, 109]
    P = [pencils.c4_pencil(j, 512, basis=b) for j, b in [pencils.c4_split("eval", 110)[i] for i in ids]]
    assert [p.m for p in P][1::2] == [0, 0]
    dev = [(fm().to_device(p.A, device()), None) for p in P]
    b = fm().FeastBatch(dev, [(p.center, p.radius, 1.0) for p in P], m0=64, q=16, precision="fp32",
                        batch_launch=mode)
    res, rcs = b.iterate([fm().to_device(pencils.start_block(4, 512, 64), device()) for _ in P])
    b.close()
    for i, p, r in zip(ids, P, res):
        ref = brute.eigenvalues_inside(p.lam, p.center, p.radius)
        assert r.converged and len(r.lam) == p.m == len(ref), (i, p.m, len(r.lam), r.iterations)
        assert r.iterations < 20, (i, r.iterations)
        if p.m:
            assert match_eigs(r.lam, ref) < 1e-9
