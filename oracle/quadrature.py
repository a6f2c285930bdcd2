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


# ---------------------------------------------------------------------------
# Glued contours (Section 5.4): the boundary is a chain of pieces, each a
# straight segment or a circular arc with a parameterisation of its own on
# [-1, 1]; the Cauchy integral over the closed curve is the sum of the pieces'
# integrals, and each is replaced by the same K-point rule.
#
# A piece is ("line", a, b) -- from a to b -- or ("arc", a, b, c) -- counter-
# clockwise about c from a to b -- with complex points.
# ---------------------------------------------------------------------------

def _arc_angles(piece):
    """Start angle and counterclockwise sweep (in (0, 2 pi)) of an arc piece."""
    _, a, b, c = piece
    th0 = math.atan2((a - c).imag, (a - c).real)
    th1 = math.atan2((b - c).imag, (b - c).real)
    d = (th1 - th0) % (2.0 * math.pi)
    return th0, d


def piece_phi(piece, t):
    """Point of a piece at parameter t in [-1, 1]."""
    t = np.asarray(t, dtype=np.float64)
    if piece[0] == "line":
        _, a, b = piece
        return a + 0.5 * (1.0 + t) * (b - a)
    _, a, b, c = piece
    th0, d = _arc_angles(piece)
    return c + abs(a - c) * np.exp(1j * (th0 + 0.5 * (1.0 + t) * d))


def piece_phi_prime(piece, t):
    """d phi / dt of a piece."""
    t = np.asarray(t, dtype=np.float64)
    if piece[0] == "line":
        _, a, b = piece
        return 0.5 * (b - a) * np.ones_like(t)
    _, a, b, c = piece
    th0, d = _arc_angles(piece)
    return 1j * 0.5 * d * abs(a - c) * np.exp(1j * (th0 + 0.5 * (1.0 + t) * d))


def glued_nodes_and_weights(pieces, rule: str, q: int):
    """(phi_j, sigma_j) of a glued contour: for each piece in turn, the K = q / len(pieces) point rule
    -- K Gauss-Legendre points, or the trapezoid with K intervals (K + 1 points) -- with weights
    w_k phi_p'(t_k) / (2 pi i); a node that two pieces share (the trapezoid's end points) is kept
    once, at its first appearance, with the two weights added."""
    P = len(pieces)
    if P < 1 or q % P:
        raise ValueError("q must be a multiple of the number of pieces")
    K = q // P
    t, w = base_rule(rule, K + 1 if rule == RULE_TRAPEZOID else K)
    zs, ss = [], []
    scale = max([1.0] + [abs(x) for pc in pieces for x in pc[1:]])
    for pc in pieces:
        z = piece_phi(pc, t)
        s = w * piece_phi_prime(pc, t) / (2j * math.pi)
        for zk, sk in zip(z, s):
            for i, zi in enumerate(zs):
                if abs(zi - zk) <= 1e-10 * scale:
                    ss[i] += sk
                    break
            else:
                zs.append(zk)
                ss.append(sk)
    if len(zs) != q:
        raise AssertionError(f"expected {q} nodes, got {len(zs)}")
    return np.array(zs), np.array(ss)


def inside_glued(mu, pieces):
    """Even-odd test: a horizontal ray from mu towards +infinity crosses the boundary an odd number
    of times.  Crossings with a segment use the half-open rule on the end points' heights; with an
    arc, the circle's two intersections with the ray's line are kept when they lie to the right of
    mu and within the arc's angular range."""
    mu = np.atleast_1d(np.asarray(mu, dtype=np.complex128))
    out = np.zeros(mu.shape, dtype=bool)
    for idx, m in np.ndenumerate(mu):
        x, y = m.real, m.imag
        cross = 0
        for pc in pieces:
            if pc[0] == "line":
                _, a, b = pc
                if (a.imag > y) != (b.imag > y):
                    xi = a.real + (y - a.imag) * (b.real - a.real) / (b.imag - a.imag)
                    if xi > x:
                        cross += 1
            else:
                _, a, b, c = pc
                r = abs(a - c)
                h = y - c.imag
                if abs(h) >= r:
                    continue
                th0, d = _arc_angles(pc)
                dx = math.sqrt(r * r - h * h)
                for xi in (c.real - dx, c.real + dx):
                    if xi <= x:
                        continue
                    off = (math.atan2(h, xi - c.real) - th0) % (2.0 * math.pi)
                    if 0.0 < off < d:
                        cross += 1
        out[idx] = cross % 2 == 1
    return out
