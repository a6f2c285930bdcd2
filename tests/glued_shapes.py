"""Glued contours used by the tests (Section 5.4's triangle, square and semicircle, and two
non-convex shapes), with closed-form membership tests and point samplers.  Inputs only: no part of
the method's arithmetic."""
import math

import numpy as np


def _piece_points(pc, t):
    """Points of a piece at parameters t in [-1, 1] (sampling only, for distances and bounds)."""
    if pc[0] == "line":
        return pc[1] + 0.5 * (1.0 + t) * (pc[2] - pc[1])
    a, b, c = pc[1], pc[2], pc[3]
    th0 = math.atan2((a - c).imag, (a - c).real)
    d = (math.atan2((b - c).imag, (b - c).real) - th0) % (2 * math.pi)
    return c + abs(a - c) * np.exp(1j * (th0 + 0.5 * (1.0 + t) * d))


TRIANGLE = [("line", 0j, 2 + 0j), ("line", 2 + 0j, 1 + 1.5j), ("line", 1 + 1.5j, 0j)]
TRIANGLE_AREA = 1.5
SQUARE = [("line", -0.5 - 0.5j, 0.5 - 0.5j), ("line", 0.5 - 0.5j, 0.5 + 0.5j),
          ("line", 0.5 + 0.5j, -0.5 + 0.5j), ("line", -0.5 + 0.5j, -0.5 - 0.5j)]
SQUARE_AREA = 1.0
# upper half of the disc |z - 0.2i| < 1.2: the arc, then the diameter back
SEMI_C, SEMI_R = 0.2j, 1.2
SEMICIRCLE = [("arc", SEMI_C + SEMI_R, SEMI_C - SEMI_R, SEMI_C), ("line", SEMI_C - SEMI_R, SEMI_C + SEMI_R)]
SEMICIRCLE_AREA = 0.5 * math.pi * SEMI_R ** 2
# disc of radius 1 without the sector |arg z| < 30 degrees: an arc sweeping 300 degrees, non-convex
MOUTH = math.pi / 6
PACMAN = [("arc", np.exp(1j * MOUTH), np.exp(-1j * MOUTH), 0j), ("line", np.exp(-1j * MOUTH), 0j),
          ("line", 0j, np.exp(1j * MOUTH))]
PACMAN_AREA = 0.5 * (2 * math.pi - 2 * MOUTH)
# L-shaped hexagon: the union of [0, 2] x [0, 1] and [0, 1] x [0, 2]
LSHAPE_V = [0j, 2 + 0j, 2 + 1j, 1 + 1j, 1 + 2j, 2j]
LSHAPE = [("line", LSHAPE_V[i], LSHAPE_V[(i + 1) % 6]) for i in range(6)]
LSHAPE_AREA = 3.0


def in_triangle(mu):
    # convex, counterclockwise: left of every edge
    v = [0j, 2 + 0j, 1 + 1.5j]
    ok = np.ones(mu.shape, bool)
    for i in range(3):
        a, b = v[i], v[(i + 1) % 3]
        ok &= ((b - a).real * (mu - a).imag - (b - a).imag * (mu - a).real) > 0
    return ok


def in_square(mu):
    return (np.abs(mu.real) < 0.5) & (np.abs(mu.imag) < 0.5)


def in_semicircle(mu):
    return (np.abs(mu - SEMI_C) < SEMI_R) & (mu.imag > SEMI_C.imag)


def in_pacman(mu):
    return (np.abs(mu) < 1) & (np.abs(np.angle(mu)) > MOUTH)


def in_lshape(mu):
    x, y = mu.real, mu.imag
    return ((x > 0) & (x < 2) & (y > 0) & (y < 1)) | ((x > 0) & (x < 1) & (y > 0) & (y < 2))


SHAPES = {"triangle": (TRIANGLE, TRIANGLE_AREA, in_triangle), "square": (SQUARE, SQUARE_AREA, in_square),
          "semicircle": (SEMICIRCLE, SEMICIRCLE_AREA, in_semicircle), "pacman": (PACMAN, PACMAN_AREA, in_pacman),
          "lshape": (LSHAPE, LSHAPE_AREA, in_lshape)}
STRAIGHT = ("triangle", "square", "lshape")


def boundary_distance(mu, pieces):
    """Distance from each point to the contour, by dense sampling (only used to keep test points
    away from the boundary)."""
    pts = np.concatenate([_piece_points(pc, np.linspace(-1, 1, 801)) for pc in pieces])
    return np.min(np.abs(mu[:, None] - pts[None, :]), axis=1)


def sample_points(pieces, seed, count=600, margin=0.03):
    g = np.random.default_rng(seed)
    pts = np.concatenate([_piece_points(pc, np.linspace(-1, 1, 65)) for pc in pieces])
    lo, hi = pts.real.min() - 0.5, pts.real.max() + 0.5
    blo, bhi = pts.imag.min() - 0.5, pts.imag.max() + 0.5
    mu = g.uniform(lo, hi, count) + 1j * g.uniform(blo, bhi, count)
    return mu[boundary_distance(mu, pieces) > margin]


def glued_spectrum(shape, n, m_in, seed, margin_in=0.1, margin_out=0.3):
    """n eigenvalues: m_in uniformly inside the shape at least margin_in from its boundary, the rest
    outside, at least margin_out from it, within twice the shape's extent."""
    pieces, _, member = SHAPES[shape]
    g = np.random.default_rng(seed)
    pts = np.concatenate([_piece_points(pc, np.linspace(-1, 1, 65)) for pc in pieces])
    mid = 0.5 * (pts.real.max() + pts.real.min()) + 0.5j * (pts.imag.max() + pts.imag.min())
    ext = max(pts.real.max() - pts.real.min(), pts.imag.max() - pts.imag.min())
    inside, outside = [], []
    while len(inside) < m_in or len(outside) < n - m_in:
        mu = mid + ext * (g.uniform(-1, 1, 512) + 1j * g.uniform(-1, 1, 512))
        d = boundary_distance(mu, pieces)
        m = member(mu)
        inside += list(mu[m & (d > margin_in)])
        outside += list(mu[~m & (d > margin_out)])
    return np.array(inside[:m_in] + outside[: n - m_in])
