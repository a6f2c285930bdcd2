"""Reduced-precision node factorisations for pinning the mixed-precision modes (test
infrastructure only; NumPy/SciPy on the host, small n).

The FP16 mode is not in the paper; it follows the reading adopted for it: a blocked right-looking
LU with partial pivoting whose working matrix and panels are FP32, and whose trailing updates take
FP16 inputs with FP32 accumulation.  Before the rounding to FP16, U12 of each step is multiplied
by 2^-e with 2^(e-1) <= max(|Re|, |Im|) over U12 < 2^e and the update is multiplied back by 2^e,
which is exact; L21 needs no scaling since partial pivoting bounds its entries.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


def _round_fp16(X):
    """Complex matrix with real and imaginary parts rounded to FP16, held in FP32."""
    return (X.real.astype(np.float16).astype(np.float32), X.imag.astype(np.float16).astype(np.float32))


def _power_of_two_exponent(mx):
    """e with 2^(e-1) <= mx < 2^e (frexp), 0 for mx == 0."""
    if mx == 0.0 or not np.isfinite(mx):
        return 0
    return math.frexp(float(mx))[1]


def factor_fp16_scaled(T, nb=64):
    """LU with partial pivoting of T (complex) with FP16-input trailing updates.

    Returns (lu, piv) in the layout of scipy.linalg.lu_factor (lu complex64; piv 0-based
    sequential interchanges), so scipy.linalg.lu_solve applies it."""
    A = np.array(T, dtype=np.complex64)
    n = A.shape[0]
    piv = np.arange(n)
    for j0 in range(0, n, nb):
        w = min(nb, n - j0)
        # panel: FP32 LU with partial pivoting of rows j0.., columns j0..j0+w-1 (cgetrf)
        panel, ppiv = scipy.linalg.lu_factor(A[j0:, j0:j0 + w], check_finite=False)
        A[j0:, j0:j0 + w] = panel
        # the panel's interchanges applied to the other columns
        for i in range(w):
            r = j0 + ppiv[i]
            piv[j0 + i] = r
            if r != j0 + i:
                for cols in (slice(0, j0), slice(j0 + w, n)):
                    tmp = A[j0 + i, cols].copy()
                    A[j0 + i, cols] = A[r, cols]
                    A[r, cols] = tmp
        if j0 + w >= n:
            break
        # U12 = L11^-1 A12 (FP32)
        L11 = np.tril(A[j0:j0 + w, j0:j0 + w], -1) + np.eye(w, dtype=np.complex64)
        U12 = scipy.linalg.solve_triangular(L11, A[j0:j0 + w, j0 + w:], lower=True, unit_diagonal=True,
                                            check_finite=False).astype(np.complex64)
        A[j0:j0 + w, j0 + w:] = U12
        # A22 -= L21 U12 with FP16 inputs (U12 scaled by 2^-e), FP32 accumulation, result times 2^e
        e = _power_of_two_exponent(max(np.abs(U12.real).max(), np.abs(U12.imag).max()))
        s = np.float32(2.0 ** -e)
        Lr, Li = _round_fp16(A[j0 + w:, j0:j0 + w])
        Ur, Ui = _round_fp16(U12 * s)
        Pr = Lr @ Ur - Li @ Ui
        Pi = Lr @ Ui + Li @ Ur
        A[j0 + w:, j0 + w:] -= (Pr + 1j * Pi).astype(np.complex64) * np.float32(2.0 ** e)
    return A, piv


def backward_error(T, lu, piv):
    """||P T - L U||_F / ||T||_F of a factorisation in lu_factor layout."""
    n = T.shape[0]
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    P = np.arange(n)
    for i in range(n):
        P[i], P[piv[i]] = P[piv[i]], P[i]
    return float(np.linalg.norm(T[P] - L.astype(np.complex128) @ U.astype(np.complex128)) / np.linalg.norm(T))
