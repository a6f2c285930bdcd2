"""Pins of the FP16-update factorisation the mixed-precision mode is checked against."""
import numpy as np
import pytest
import scipy.linalg

import pencils
from oracle import feast, lowprec


def rand_T(n, seed, shift=2.0):
    g = np.random.default_rng(seed)
    return pencils.complex_gaussian(g, (n, n)) + shift * np.sqrt(n) * np.eye(n)


def test_single_panel_equals_lapack():
    """With one panel (nb >= n) there is no trailing update: the factorisation is LAPACK's FP32
    partial-pivoting LU exactly (same pivots, same factors)."""
    T = rand_T(50, 1, shift=0.0)
    lu, piv = lowprec.factor_fp16_scaled(T, nb=64)
    lu32, piv32 = scipy.linalg.lu_factor(T.astype(np.complex64))
    assert np.array_equal(piv, piv32)
    assert np.array_equal(lu, lu32)


def test_backward_error_is_fp16_level():
    """FP16 inputs to the updates put the backward error well above FP32 LU and at most a small
    multiple of u16 = 2^-11 (several trailing updates at n = 256, nb = 64)."""
    T = rand_T(256, 2, shift=0.0)
    e16 = lowprec.backward_error(T, *lowprec.factor_fp16_scaled(T))
    e32 = lowprec.backward_error(T, *scipy.linalg.lu_factor(T.astype(np.complex64)))
    assert e32 < 3e-6
    assert 30 * e32 < e16 < 20 * 2.0 ** -11


def test_scaling_is_exact_and_needed():
    """Scaling T by 2^20 scales U by 2^20 and leaves L and the pivots unchanged, bit for bit; without
    the power-of-two scale of U12 the FP16 inputs overflow (a planted mistake in the oracle)."""
    T = rand_T(150, 3, shift=0.0)
    lu, piv = lowprec.factor_fp16_scaled(T)
    lu2, piv2 = lowprec.factor_fp16_scaled(T * 2.0 ** 20)
    assert np.array_equal(piv, piv2)
    assert np.array_equal(np.tril(lu2, -1), np.tril(lu, -1))
    assert np.array_equal(np.triu(lu2), np.triu(lu) * np.float32(2.0 ** 20))
    saved = lowprec._power_of_two_exponent
    try:
        lowprec._power_of_two_exponent = lambda mx: 0
        with np.errstate(all="ignore"):
            bad, _ = lowprec.factor_fp16_scaled(T * 2.0 ** 20)
        assert not np.all(np.isfinite(bad))
    finally:
        lowprec._power_of_two_exponent = saved


def test_refinement_with_fp16_factors_reaches_fp64():
    """FP64 refinement with the FP16-update factors converges to the FP64 solution when kappa(T) u16
    is well below 1, taking more sweeps than with FP32 factors."""
    T = rand_T(200, 4)
    rhs = pencils.complex_gaussian(np.random.default_rng(5), (200, 6))
    ref = np.linalg.solve(T, rhs)
    kappa = np.linalg.cond(T)
    assert kappa < 20
    y16, s16, _ = feast.solve_refined(T, rhs, factor=lowprec.factor_fp16_scaled, ir_max=30)
    y32, s32, _ = feast.solve_refined(T, rhs)
    for y in (y16, y32):
        assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 50 * kappa * feast.U64 * np.sqrt(200)
    assert s16 > s32
