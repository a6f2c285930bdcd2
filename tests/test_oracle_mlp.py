"""Pins of the reference perceptron: finite differences, the first Adam step in closed form, and a
regression it must learn."""
import numpy as np

from oracle import mlp


def small(seed=0, n_in=5, hidden=7):
    g = np.random.default_rng(seed)
    return mlp.init_params(g, n_in, hidden), g.standard_normal((11, n_in)), g.standard_normal(11)


def test_gradients_match_central_differences():
    P, X, t = small()
    y, cache = mlp.forward(P, X)
    G = mlp.flatten(mlp.backward(P, cache, y, t))
    v = mlp.flatten(P)
    h = 1e-6
    fd = np.zeros_like(v)
    for i in range(len(v)):
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        fd[i] = (mlp.mse(mlp.forward(mlp.unflatten(vp, 5, 7), X)[0], t) -
                 mlp.mse(mlp.forward(mlp.unflatten(vm, 5, 7), X)[0], t)) / (2 * h)
    assert np.linalg.norm(G - fd) < 1e-7 * np.linalg.norm(fd)


def test_relu_and_layers_by_hand():
    """One hidden unit per layer: y = w3 relu(w2 relu(w1 x + b1) + b2) + b3 written out."""
    P = {"W1": np.array([[2.0]]), "b1": np.array([-1.0]), "W2": np.array([[-3.0]]), "b2": np.array([4.0]),
         "W3": np.array([[0.5]]), "b3": np.array([0.25])}
    X = np.array([[0.0], [1.0], [3.0]])
    y, _ = mlp.forward(P, X)
    expect = [0.5 * max(-3 * max(2 * x - 1, 0) + 4, 0) + 0.25 for x in (0.0, 1.0, 3.0)]
    assert np.allclose(y, expect)


def test_first_adam_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so every parameter moves by
    -lr g / (|g| + eps)."""
    P, X, t = small(1)
    y, cache = mlp.forward(P, X)
    G = mlp.backward(P, cache, y, t)
    v0, g = mlp.flatten(P), mlp.flatten(G)
    P1 = mlp.adam_step({k: v.copy() for k, v in P.items()}, G, mlp.adam_init(P), 1, lr=0.01)
    assert np.allclose(mlp.flatten(P1), v0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_adam_learns_a_smooth_regression():
    g = np.random.default_rng(2)
    X = g.uniform(-1, 1, size=(256, 3))
    t = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]
    P = mlp.init_params(g, 3, 32)
    st = mlp.adam_init(P)
    first = mlp.mse(mlp.forward(P, X)[0], t)
    for step in range(1, 401):
        y, cache = mlp.forward(P, X)
        mlp.adam_step(P, mlp.backward(P, cache, y, t), st, step, lr=1e-2)
    assert mlp.mse(mlp.forward(P, X)[0], t) < 0.05 * first
