"""The definition the iteration converges to (paper Section 2).  Test infrastructure only.

The targets are the eigenvalues of the pencil (A, B) strictly inside the
domain (none lie on its boundary), m of them, with right eigenvectors X_C.
This module computes them by brute force: every generalized eigenvalue by QZ
(LAPACK zggev through SciPy), then the inside test.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .quadrature import inside


def all_eigenvalues(A, B=None):
    """Every eigenvalue of A x = lambda B x (QZ)."""
    if B is None:
        return scipy.linalg.eigvals(A)
    return scipy.linalg.eigvals(A, B)


def eigenvalues_inside(lam, c, R, a=1.0):
    lam = np.asarray(lam)
    return lam[inside(lam, c, R, a)]


def count_inside(lam, c, R, a=1.0):
    return int(np.count_nonzero(inside(lam, c, R, a)))


def radius_for_count(lam, c, m_target):
    """Circle radius in the middle of the gap between the m-th and (m+1)-th nearest eigenvalue to c.

    Returns (R, lower, upper) where lower/upper are the two distances."""
    d = np.sort(np.abs(np.asarray(lam) - c))
    lo, hi = float(d[m_target - 1]), float(d[m_target])
    return 0.5 * (lo + hi), lo, hi


def eigenpair_null_vector(A, B, lam):
    """Right eigenvector for an eigenvalue lam: the right singular vector of A - lam B with the
    smallest singular value (tiny n only)."""
    M = A - lam * (np.eye(A.shape[0]) if B is None else B)
    _, _, Vh = np.linalg.svd(M)
    return Vh[-1].conj()
