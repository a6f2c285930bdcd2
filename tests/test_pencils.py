"""The seeded input generators: the batched workload's factored construction has the spectrum it
prescribes and the distribution of the clipped complex Gaussian basis it stands for."""
import numpy as np
import pytest
import scipy.linalg
from scipy.optimize import linear_sum_assignment

import pencils


def test_chi_model_singular_values_match_gaussian_svd():
    """Mean sorted singular values of the chi bidiagonal model agree with those of explicit complex
    Gaussian matrices within a few standard errors (400 draws each, n = 48)."""
    g = np.random.default_rng(11)
    n, reps = 48, 400
    a = np.array([pencils.gaussian_singular_values(g, n) for _ in range(reps)])
    b = np.array([np.linalg.svd(pencils.complex_gaussian(g, (n, n)), compute_uv=False) for _ in range(reps)])
    se = np.sqrt(a.var(axis=0) / reps + b.var(axis=0) / reps)
    assert np.all(np.abs(a.mean(axis=0) - b.mean(axis=0)) < 5 * se + 1e-12)
    # second moment: E sum s_i^2 = E ||G||_F^2 = n^2
    assert abs(np.mean(np.sum(a * a, axis=1)) / n ** 2 - 1) < 0.02


def test_haar_unitary_is_unitary_and_phase_fixed():
    g = np.random.default_rng(3)
    Q = pencils.haar_unitary(pencils.complex_gaussian(g, (40, 40)))
    assert np.allclose(Q.conj().T @ Q, np.eye(40), atol=1e-13)


@pytest.mark.parametrize("n,m", [(64, 3), (200, 16), (331, 25)])
def test_batched_pencil_has_prescribed_spectrum(n, m):
    P = pencils.c2_pencil(5, n, m)
    ev = scipy.linalg.eigvals(P.A, P.B)
    C = np.abs(ev[:, None] - P.lam[None, :])
    r, c = linear_sum_assignment(C)
    assert C[r, c].max() < 1e-10 * np.abs(P.lam).max()
    assert np.sum(np.abs(P.lam) < 1.0) == m
    assert P.m0 == (16 if m <= 16 else 32)
    # B Hermitian with spectrum near 1
    assert np.allclose(P.B, P.B.conj().T)
    assert np.linalg.cond(P.B) < 1.5


def test_batched_pencil_torch_path_matches_numpy():
    torch = pytest.importorskip("torch")
    P = pencils.c2_pencil(3, 150, 9)
    Q = pencils.c2_pencil(3, 150, 9, device="cpu")
    assert Q.A.stride() == (1, 150)
    assert np.abs(Q.A.numpy() - P.A).max() < 1e-12 * np.abs(P.A).max()
    assert np.array_equal(Q.B.numpy(), P.B)


def test_real_pencil_has_real_entries_and_the_stated_spectrum():
    import scipy.linalg
    from tests.gpu_common import match_eigs
    A, B, lam = pencils.real_pencil(np.random.default_rng(3), 61, 4, 3)
    assert np.all(A.imag == 0) and np.all(B.imag == 0)
    assert np.sum(np.abs(lam) < 0.8) == 11
    assert match_eigs(scipy.linalg.eigvals(A, B), lam) < 1e-9
