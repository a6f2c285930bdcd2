"""Pins of the brute-force helpers: shift-invert Arnoldi agrees with full QZ on small pencils."""
import numpy as np

import pencils
from oracle import brute


def test_nearest_eigenvalues_match_qz():
    P = pencils.c1(n=300)
    full = brute.all_eigenvalues(P.A, P.B)
    full = full[np.argsort(np.abs(full - P.center))]
    near = brute.nearest_eigenvalues(P.A, P.B, P.center, 30)
    assert np.abs(near - full[:30]).max() < 1e-11


def test_nearest_eigenvalues_prescribed():
    P = pencils.c0(n=120, m=7)
    near = brute.nearest_eigenvalues(P.A, None, 0j, 7)
    ref = P.lam[np.argsort(np.abs(P.lam))][:7]
    assert np.abs(near - ref).max() < 1e-10


def test_widest_gap_radius():
    lam = np.array([0.1, 0.2, 0.3, 0.31, 0.5, 0.52, 0.6])
    R, m, lo, hi = brute.widest_gap_radius(lam, 0.0, 4, window=2)
    assert m == 4 and lo == 0.31 and hi == 0.5 and abs(R - 0.405) < 1e-15
    assert brute.count_inside(lam, 0.0, R) == 4
