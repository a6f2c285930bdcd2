"""Pins of the oracle's contour, quadrature and filter (paper Section 3) against closed forms.

None of these retype the oracle's formula: the trapezoid filter on a circle is
checked against its closed form 1/(1 - w^q) (a roots-of-unity identity), the
base rules against exact polynomial integrals, the folded rule against a
fine periodic trapezoid of the unfolded Cauchy integral, and the indicator
eta(r) against its closed form for the trapezoid."""
import math

import numpy as np
import pytest

from oracle import quadrature as Q

TR, GL = Q.RULE_TRAPEZOID, Q.RULE_GAUSS_LEGENDRE


def rng(seed=0):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("q", [2, 4, 8, 16, 24, 32])
@pytest.mark.parametrize("c,R", [(0j, 1.0), (0.5 + 0.2j, 0.3), (-2 + 1j, 3.5)])
def test_trapezoid_circle_closed_form(q, c, R):
    z, s = Q.nodes_and_weights(c, R, 1.0, TR, q)
    g = rng(q)
    mu = c + R * (g.uniform(0, 2.5, 50) * np.exp(2j * np.pi * g.random(50)))
    w = (mu - c) / R
    expect = 1.0 / (1.0 - w ** q)
    got = Q.rho(mu, z, s)
    assert np.allclose(got, expect, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("rule", [TR, GL])
@pytest.mark.parametrize("q", [4, 8, 16, 24])
@pytest.mark.parametrize("a", [1.0, 0.5, 2.0])
def test_center_value_is_one(rule, q, a):
    """rho(c) = 1 for any rule with weights summing to 2 on a circle; for an ellipse it is the
    quadrature of the constant 1/(2 pi i) phi'/(phi - c), which is exact only for a = 1."""
    z, s = Q.nodes_and_weights(0.3 - 0.1j, 0.7, a, rule, q)
    val = Q.rho(np.array([0.3 - 0.1j]), z, s)[0]
    if a == 1.0:
        assert abs(val - 1.0) < 1e-13
    else:
        assert abs(val - 1.0) < 0.05 * (16 / q) ** 2


@pytest.mark.parametrize("q", [4, 8, 16, 32])
def test_node_counts_and_contour(q):
    for rule, K in [(TR, q // 2 + 1), (GL, q // 2)]:
        assert Q.points_per_half(rule, q) == K
        z, s = Q.nodes_and_weights(1 + 1j, 2.0, 0.5, rule, q)
        assert len(z) == q and len(set(np.round(z, 12))) == q
        x, y = (z - (1 + 1j)).real / 2.0, (z - (1 + 1j)).imag / (0.5 * 2.0)
        assert np.allclose(x * x + y * y, 1.0, atol=1e-14)


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8, 12])
def test_gauss_legendre_exactness(K):
    t, w = Q.base_rule(GL, K)
    assert np.all(w > 0) and np.all(np.abs(t) < 1)
    for j in range(2 * K):
        exact = 0.0 if j % 2 else 2.0 / (j + 1)
        assert abs(np.sum(w * t ** j) - exact) < 1e-13


@pytest.mark.parametrize("K", [2, 3, 9, 17])
def test_trapezoid_base_rule(K):
    t, w = Q.base_rule(TR, K)
    assert t[0] == -1.0 and t[-1] == 1.0
    assert abs(w.sum() - 2.0) < 1e-15
    assert abs(np.sum(w * t)) < 1e-15                     # exact for linear functions
    # composite trapezoid error for t^2: h^2/6 * (f'(1) - f'(-1)) / 2 ... exact value 2/3 + h^2/3
    h = 2.0 / (K - 1)
    assert abs(np.sum(w * t * t) - (2.0 / 3.0 + h * h / 3.0)) < 1e-14


def _cauchy_unfolded(mu, c, R, a, N=4000):
    """(1/2 pi i) integral over [-1, 3] of phi'(t)/(phi(t) - mu), periodic trapezoid with N points."""
    t = -1.0 + 4.0 * np.arange(N) / N
    th = 0.5 * np.pi * (1 + t)
    ph = c + R * (np.cos(th) + 1j * a * np.sin(th))
    dph = R * 0.5 * np.pi * (-np.sin(th) + 1j * a * np.cos(th))
    return (4.0 / N) * np.sum(dph / (ph - mu)) / (2j * np.pi)


@pytest.mark.parametrize("rule", [TR, GL])
@pytest.mark.parametrize("a", [1.0, 0.4, 1.7])
def test_fold_converges_to_cauchy_integral(rule, a):
    """The folded rule converges to the unfolded Cauchy integral (1 inside, 0 outside) as q grows."""
    c, R = 0.2 + 0.1j, 1.3
    z, s = Q.nodes_and_weights(c, R, a, rule, 128)
    for rel, expect in [(0.3, 1.0), (0.5, 1.0), (1.8, 0.0), (3.0, 0.0)]:
        for ang in [0.1, 1.3, 2.9, 4.4]:
            mu = c + rel * R * (math.cos(ang) + 1j * a * math.sin(ang))
            ref = _cauchy_unfolded(mu, c, R, a)
            assert abs(ref - expect) < 1e-9
            assert abs(Q.rho(np.array([mu]), z, s)[0] - expect) < 1e-6


@pytest.mark.parametrize("q", [8, 16, 24])
def test_eta_trapezoid_closed_form(q):
    r_in = np.array([0.0, 0.3, 0.8, 0.95, 0.99])
    r_out = np.array([1.01, 1.2, 1.5, 3.0])
    assert np.allclose(Q.eta(r_in, TR, q), 1.0 / (1.0 + r_in ** q), rtol=1e-6)
    assert np.allclose(Q.eta(r_out, TR, q), 1.0 / (r_out ** q - 1.0), rtol=1e-6)


def test_trapezoid_beats_gauss_legendre_off_axis():
    """Section 3: a K-point GL and a (K+1)-point TR cost the same (2K systems); for the circle
    the trapezoid attenuates more strongly just outside (Figure eta circle GL vs TR)."""
    q = 16
    r = np.array([1.2, 1.5])
    assert np.all(Q.eta(r, TR, q) < Q.eta(r, GL, q))


def test_inside_strict():
    assert Q.inside(np.array([0.5]), 0, 1.0)[0]
    assert not Q.inside(np.array([1.0]), 0, 1.0)[0]
    assert Q.inside(np.array([0.45j]), 0, 1.0, 0.5)[0]
    assert not Q.inside(np.array([0.55j]), 0, 1.0, 0.5)[0]


@pytest.mark.parametrize("rule", [TR, GL])
@pytest.mark.parametrize("q", [8, 16, 24, 32])
def test_filter_gain_is_at_least_one_half_inside(rule, q):
    """|rho| > 1/2 everywhere inside the circle (for the trapezoid, |1 - w^q| < 2 when |w| < 1), the
    bound behind the library's empty-contour rule in its low-precision modes: a Ritz vector that has
    captured an eigenvector of an eigenvalue inside is amplified by at least 1/2, ten times its
    threshold of 0.05; eigenvalues 1.5 radii or more from the centre stay below that threshold for
    q >= 16 (at q = 8 the Gauss-Legendre filter does not, which only keeps the strict rule in force)."""
    z, s = Q.nodes_and_weights(0.3 + 0.2j, 0.8, 1.0, rule, q)
    g = rng(q + 100)
    th = 2 * np.pi * g.random(20000)
    w_in = np.sqrt(g.random(20000)) * 0.999 * np.exp(1j * th)
    assert np.abs(Q.rho(0.3 + 0.2j + 0.8 * w_in, z, s)).min() > 0.5
    w_out = (1.5 + 3.5 * g.random(20000)) * np.exp(1j * th)
    out = np.abs(Q.rho(0.3 + 0.2j + 0.8 * w_out, z, s)).max()
    if q >= 16:
        assert out < 0.05 / 3
