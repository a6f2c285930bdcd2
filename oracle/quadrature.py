"""Contour, quadrature and rational filter (paper Section 3).  Test infrastructure only.

* The contour is the ellipse of eqn:ellipses,
      phi(t) = c + R (cos(pi/2 (1+t)) + i a sin(pi/2 (1+t))),  t in [-1, 3],
  traversed counter-clockwise; horizontal semi-axis R, vertical semi-axis aR.
* The Cauchy integral of eqn:cauchy_contour is split at t = 1 and the second
  half folded onto [-1, 1] with t~ = 2 - t (eqn:pi).  A K-point rule (t_k, w_k)
  on [-1, 1] then gives eqn:quadrature_for_pi,
      rho(mu) = sum_k w_k / (2 pi i) (phi'(t_k)/(phi(t_k) - mu) + phi'(t~_k)/(phi(t~_k) - mu))
              = sum_j sigma_j / (phi_j - mu),
  with q = 2K nodes when +-1 are not rule nodes (Gauss-Legendre) and
  q = 2(K - 1) when they are (trapezoid): the coincident nodes at t = 1 = 2 - 1
  and at t = -1 ~ t = 3 merge (their weights add).
"""
from __future__ import annotations

import math

import numpy as np

RULE_TRAPEZOID = "trapezoid"
RULE_GAUSS_LEGENDRE = "gauss-legendre"


def phi(t, c, R, a):
    """Point of the elliptic contour at parameter t (eqn:ellipses)."""
    th = 0.5 * math.pi * (1.0 + np.asarray(t, dtype=np.float64))
    return c + R * (np.cos(th) + 1j * a * np.sin(th))


def phi_prime(t, R, a):
    """d phi / dt."""
    th = 0.5 * math.pi * (1.0 + np.asarray(t, dtype=np.float64))
    return R * 0.5 * math.pi * (-np.sin(th) + 1j * a * np.cos(th))


def base_rule(rule: str, K: int):
    """K-point rule (t_k, w_k) on [-1, 1] with positive weights summing to 2."""
    if rule == RULE_TRAPEZOID:
        if K < 2:
            raise ValueError("trapezoid needs K >= 2")
        t = -1.0 + 2.0 * np.arange(K) / (K - 1)
        w = np.full(K, 2.0 / (K - 1))
        w[0] *= 0.5
        w[-1] *= 0.5
        return t, w
    if rule == RULE_GAUSS_LEGENDRE:
        t, w = np.polynomial.legendre.leggauss(K)
        return t, w
    raise ValueError(rule)


def points_per_half(rule: str, q: int) -> int:
    """K such that the folded rule yields q distinct nodes (q = 2K or q = 2(K - 1))."""
    if q < 2 or q % 2:
        raise ValueError("q must be even and >= 2")
    return q // 2 + 1 if rule == RULE_TRAPEZOID else q // 2


def nodes_and_weights(c: complex, R: float, a: float, rule: str, q: int):
    """(phi_j, sigma_j), j = 1..q, of eqn:quadrature_for_pi, coincident nodes merged.

    Order: the nodes of the first half (t_k increasing), then the folded half
    (t~_k = 2 - t_k, t_k decreasing), with duplicates dropped after merging."""
    K = points_per_half(rule, q)
    t, w = base_rule(rule, K)
    ts = np.concatenate([t, (2.0 - t)[::-1]])
    ws = np.concatenate([w, w[::-1]])
    z = phi(ts, c, R, a)
    s = ws * phi_prime(ts, R, a) / (2j * math.pi)
    # merge coincident nodes: t = 1 appears in both halves; t = -1 and t = 3 are the same point
    zs, ss = [], []
    tol = 1e-12 * max(1.0, abs(c) + R * max(1.0, a))
    for zk, sk in zip(z, s):
        for i, zi in enumerate(zs):
            if abs(zi - zk) <= tol:
                ss[i] += sk
                break
        else:
            zs.append(zk)
            ss.append(sk)
    zs = np.array(zs)
    ss = np.array(ss)
    if len(zs) != q:
        raise AssertionError(f"expected {q} nodes, got {len(zs)}")
    return zs, ss


def rho(mu, z, sigma):
    """Rational filter rho(mu) = sum_j sigma_j / (z_j - mu) (eqn:quadrature_for_pi)."""
    mu = np.asarray(mu, dtype=np.complex128)
    out = np.zeros(mu.shape, dtype=np.complex128)
    for zk, sk in zip(z, sigma):
        out += sk / (zk - mu)
    return out


def inside(mu, c, R, a=1.0):
    """Strictly inside the ellipse with semi-axes R (horizontal) and aR (vertical)."""
    d = np.asarray(mu) - c
    return (d.real / R) ** 2 + (d.imag / (a * R)) ** 2 < 1.0


def eta(r_values, rule: str, q: int, a: float = 1.0, samples: int = 2048):
    """Indicator eta(r) of Section 3: min |rho_ref| on the level curve r phi for r < 1, max for r > 1.

    rho_ref is the filter of the reference ellipse (center 0, R = 1, same a)."""
    z, s = nodes_and_weights(0j, 1.0, a, rule, q)
    tt = np.linspace(-1.0, 3.0, samples, endpoint=False)
    out = []
    for r in np.atleast_1d(r_values):
        mu = r * (phi(tt, 0j, 1.0, a))
        v = np.abs(rho(mu, z, s))
        out.append(v.min() if r < 1.0 else v.max())
    return np.array(out)
