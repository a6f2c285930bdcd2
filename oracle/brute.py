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


def eigenpair_null_vector(A, B, lam):
    """Right eigenvector for an eigenvalue lam: the right singular vector of A - lam B with the
    smallest singular value (tiny n only)."""
    M = A - lam * (np.eye(A.shape[0]) if B is None else B)
    _, _, Vh = np.linalg.svd(M)
    return Vh[-1].conj()


def nearest_eigenvalues(A, B, c, k, tol=0.0):
    """The k eigenvalues of (A, B) nearest to c, by shift-invert Arnoldi (ARPACK through SciPy):
    the largest-modulus eigenvalues nu of (A - c B)^-1 B give lambda = c + 1/nu.

    For pencils too large for QZ on the host (n = 4096, 8192); pinned against QZ on small pencils."""
    import scipy.sparse.linalg as sla
    n = A.shape[0]
    Bm = np.eye(n, dtype=np.complex128) if B is None else B
    lu = scipy.linalg.lu_factor(A - c * Bm)

    def mv(x):
        return scipy.linalg.lu_solve(lu, Bm @ x)

    op = sla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    ncv = min(n - 1, max(2 * k + 1, k + 40))
    nu = sla.eigs(op, k=k, which="LM", ncv=ncv, tol=tol, return_eigenvectors=False, maxiter=10 * n)
    lam = c + 1.0 / nu
    return lam[np.argsort(np.abs(lam - c))]


def widest_gap_radius(lam, c, m_target, window=6):
    """Circle radius for a count near m_target: among counts m_target-window..m_target+window pick the
    one whose gap d_(m+1) - d_m, relative to d_m, is widest, and return (R, m, d_m, d_(m+1)) with R
    the middle of that gap."""
    d = np.sort(np.abs(np.asarray(lam) - c))
    best = None
    for m in range(max(1, m_target - window), min(len(d) - 1, m_target + window) + 1):
        g = (d[m] - d[m - 1]) / d[m - 1]
        if best is None or g > best[0]:
            best = (g, m)
    m = best[1]
    return 0.5 * (d[m - 1] + d[m]), m, float(d[m - 1]), float(d[m])
