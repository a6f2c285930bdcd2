"""Pins of the oracle's filters and FEAST iterations against exact identities and brute force.

* eqn:quadf_surM: on a pencil with prescribed spectrum (B^-1 A = V L V^-1),
  rho(M) U = V rho(L) V^-1 U, evaluated with the closed-form trapezoid filter
  1/(1 - w^q) (not with the node sums).
* eqn:quadf_surMconj: the left filter equals Y conj(rho(L)) X^H B^H V with
  X = V, Y = B^-H V^-H.
* R-FEAST / Bi-FEAST converge to exactly the prescribed eigenvalues inside the
  contour (the definition of Section 2), with the right count, and at the rate
  the convergence properties of Section 4 predict.
* Planted mistakes (conjugate dropped, weight sign flipped, B dropped, fold
  not applied) each break at least one pin.
"""
import numpy as np
import pytest
import scipy.linalg

import pencils
from oracle import brute, feast
from oracle import quadrature as Q

TR, GL = Q.RULE_TRAPEZOID, Q.RULE_GAUSS_LEGENDRE


def small_pencil(n=40, m=5, with_B=False, seed=7, r_in=1.5):
    g = np.random.default_rng(seed)
    lam = pencils.prescribed_spectrum(g, n, m, r_in=r_in)
    B = None
    if with_B:
        H = pencils.complex_gaussian(g, (n, n))
        B = np.eye(n) + 0.1 * (H + H.conj().T) / (2 * np.sqrt(n)) + 0.05 * pencils.complex_gaussian(g, (n, n)) / np.sqrt(n)
    V = pencils.clipped_gaussian_basis(g, n, 1e2)
    A = (V * lam) @ np.linalg.inv(V)
    if B is not None:
        A = B @ A
    return A, B, lam, V


def closed_form_rho_tr(lam, c, R, q):
    return 1.0 / (1.0 - ((lam - c) / R) ** q)


@pytest.mark.parametrize("with_B", [False, True])
@pytest.mark.parametrize("q", [8, 16])
def test_right_filter_closed_form(with_B, q):
    A, B, lam, V = small_pencil(with_B=with_B)
    c, R = 0.1 + 0.05j, 1.05
    z, s = Q.nodes_and_weights(c, R, 1.0, TR, q)
    U = pencils.complex_gaussian(np.random.default_rng(1), (A.shape[0], 6))
    got = feast.filter_right(feast.factor_nodes(A, B, z), s, B, U)
    expect = V @ (closed_form_rho_tr(lam, c, R, q)[:, None] * np.linalg.solve(V, U))
    assert np.linalg.norm(got - expect) / np.linalg.norm(expect) < 1e-11


@pytest.mark.parametrize("with_B", [False, True])
def test_left_filter_closed_form(with_B):
    A, B, lam, V = small_pencil(with_B=with_B, seed=11)
    n = A.shape[0]
    c, R, q = -0.05j, 0.95, 16
    z, s = Q.nodes_and_weights(c, R, 1.0, TR, q)
    Vin = pencils.complex_gaussian(np.random.default_rng(2), (n, 5))
    got = feast.filter_left(feast.factor_nodes(A, B, z), s, B, Vin)
    Bm = np.eye(n) if B is None else B
    X = V
    Y = np.linalg.inv(Bm.conj().T) @ np.linalg.inv(V).conj().T
    assert np.allclose(Y.conj().T @ Bm @ X, np.eye(n), atol=1e-9)
    expect = Y @ (np.conj(closed_form_rho_tr(lam, c, R, q))[:, None] * (X.conj().T @ (Bm.conj().T @ Vin)))
    assert np.linalg.norm(got - expect) / np.linalg.norm(expect) < 1e-11


def test_gauss_legendre_filter_matches_scalar_filter_on_spectrum():
    A, B, lam, V = small_pencil(with_B=True, seed=3)
    c, R, q = 0j, 1.0, 16
    z, s = Q.nodes_and_weights(c, R, 1.0, GL, q)
    U = pencils.complex_gaussian(np.random.default_rng(4), (A.shape[0], 4))
    got = feast.filter_right(feast.factor_nodes(A, B, z), s, B, U)
    expect = V @ (Q.rho(lam, z, s)[:, None] * np.linalg.solve(V, U))
    assert np.linalg.norm(got - expect) / np.linalg.norm(expect) < 1e-11


def test_node_solves_backward_error():
    A, B, lam, V = small_pencil(n=60, with_B=True)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, TR, 8)
    rhs = pencils.complex_gaussian(np.random.default_rng(5), (60, 3))
    lus = feast.factor_nodes(A, B, z)
    for zk, Yk, Yh in zip(z, feast.solve_nodes(lus, rhs), feast.solve_nodes(lus, rhs, conj_trans=True)):
        T = zk * B - A
        assert np.allclose(Yk, np.linalg.solve(T, rhs), rtol=1e-10, atol=1e-12)
        assert np.allclose(Yh, np.linalg.solve(T.conj().T, rhs), rtol=1e-10, atol=1e-12)
        assert np.linalg.norm(T @ Yk - rhs) <= 1e-13 * np.linalg.norm(T, 1) * np.linalg.norm(Yk) * 60


def match_eigs(got, ref):
    """Optimal assignment of two eigenvalue sets; returns the max relative error."""
    from scipy.optimize import linear_sum_assignment
    assert len(got) == len(ref)
    C = np.abs(got[:, None] - ref[None, :]) / np.abs(ref)[None, :]
    r, c = linear_sum_assignment(C)
    return C[r, c].max()


def test_brute_force_recovers_prescribed_spectrum():
    A, B, lam, V = small_pencil(n=50, with_B=True)
    ev = brute.all_eigenvalues(A, B)
    assert match_eigs(ev, lam) < 1e-9
    assert brute.count_inside(ev, 0, 1.0) == 5


@pytest.mark.parametrize("algo", ["R", "Bi"])
def test_feast_c0_converges_to_definition(algo):
    P = pencils.c0()
    U0 = pencils.start_block(0, P.n, P.m0)
    run = feast.rfeast if algo == "R" else feast.bifeast
    r = run(P.A, P.B, P.center, P.radius, P.aspect, P.q, U0)
    assert r.converged and r.iters <= 6
    ref = brute.eigenvalues_inside(P.lam, P.center, P.radius)
    assert r.m == len(ref) == 10
    assert match_eigs(r.lam, ref) < 1e-10
    assert r.resid.max() <= 1e-10
    # eigenvectors: the null vectors of A - lam I, phase free
    for j in range(r.m):
        x = brute.eigenpair_null_vector(P.A, P.B, r.lam[j])
        assert 1 - abs(np.vdot(x, r.X[:, j])) < 1e-9
    if algo == "Bi":
        assert r.resid_left.max() < 1e-8


@pytest.mark.parametrize("algo", ["R", "Bi"])
def test_feast_generalized_pencil(algo):
    A, B, lam, V = small_pencil(n=80, m=6, with_B=True, seed=21)
    U0 = pencils.complex_gaussian(np.random.default_rng(9), (80, 10))
    run = feast.rfeast if algo == "R" else feast.bifeast
    r = run(A, B, 0j, 1.0, 1.0, 16, U0)
    ref = brute.eigenvalues_inside(lam, 0, 1.0)
    assert r.converged and r.m == len(ref) == 6
    assert match_eigs(r.lam, ref) < 1e-10


def test_feast_ellipse_and_gauss_legendre():
    A, B, lam, V = small_pencil(n=60, m=8, seed=5)
    # an ellipse with semi-axes 1 and 0.7 that holds some of the inside eigenvalues
    a = 0.7
    ref = brute.eigenvalues_inside(lam, 0, 1.0, a)
    U0 = pencils.complex_gaussian(np.random.default_rng(3), (60, len(ref) + 4))
    r = feast.rfeast(A, B, 0j, 1.0, a, 16, U0, rule=GL, max_iter=40)
    assert r.converged and r.m == len(ref)
    assert match_eigs(r.lam, ref) < 1e-10


def predicted_rate(lam, c, R, q, p, m):
    """log10 |gamma_{p+1} / gamma_m| with gamma = closed-form trapezoid rho on the spectrum."""
    g = np.sort(np.abs(closed_form_rho_tr(lam, c, R, q)))[::-1]
    return np.log10(g[p] / g[m - 1])


def test_rfeast_rate_matches_prediction():
    """Section 4, property 2: residuals fall like eps^k, eps = |gamma_{p+1}/gamma_m|."""
    n, m, p, q = 120, 6, 8, 8
    A, B, lam, V = small_pencil(n=n, m=m, seed=33, r_in=1.08)
    pred = predicted_rate(lam, 0, 1.0, q, p, m)
    assert -2.0 < pred < -0.3
    U0 = pencils.complex_gaussian(np.random.default_rng(8), (n, p))
    r = feast.rfeast(A, B, 0j, 1.0, 1.0, q, U0, tol=1e-13, max_iter=25)
    res = np.array([h["res_paper"] for h in r.history])
    ok = np.isfinite(res) & (res > 1e-12) & (res < 1e-3)
    k = np.arange(1, len(res) + 1)[ok]
    slope = np.polyfit(k, np.log10(res[ok]), 1)[0]
    assert len(k) >= 4
    assert abs(slope - pred) < 0.35 * abs(pred) + 0.1


def test_bifeast_eigenvalues_converge_twice_as_fast():
    """Section 4, property 3: Bi-FEAST eigenvalue errors fall like eps^(2k), residuals like eps^k."""
    n, m, p, q = 120, 6, 8, 8
    A, B, lam, V = small_pencil(n=n, m=m, seed=33, r_in=1.08)
    ref = brute.eigenvalues_inside(lam, 0, 1.0)
    U0 = pencils.complex_gaussian(np.random.default_rng(8), (n, p))
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, TR, q)
    lus = feast.factor_nodes(A, B, z)

    def eig_errors(run):
        errs = {}
        for it in range(2, 10):
            r = run(A, B, 0j, 1.0, 1.0, q, U0, max_iter=it, tol=0.0, lus=lus)
            # distance from each target eigenvalue to the nearest Ritz value
            d = np.abs(ref[:, None] - r.ritz[None, :]).min(axis=1) / np.abs(ref)
            errs[it] = d.max()
        return errs

    er = eig_errors(feast.rfeast)
    eb = eig_errors(feast.bifeast)
    ks = [k for k in er if 1e-12 < eb[k] < 1e-3 and 1e-12 < er[k] < 1e-3]
    assert len(ks) >= 3
    slope_r = np.polyfit(ks, np.log10([er[k] for k in ks]), 1)[0]
    slope_b = np.polyfit(ks, np.log10([eb[k] for k in ks]), 1)[0]
    assert slope_r < -0.3
    assert slope_b < 1.5 * slope_r      # both negative: Bi-FEAST at least 1.5x steeper


def test_refinement_reaches_fp64_solution():
    A, B, lam, V = small_pencil(n=100, with_B=True, seed=2)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, TR, 8)
    rhs = pencils.complex_gaussian(np.random.default_rng(6), (100, 4))
    for zk in z[:3]:
        T = zk * B - A
        Y, sweeps, norms = feast.solve_refined(T, rhs)
        Y64 = np.linalg.solve(T, rhs)
        kappa = np.linalg.cond(T)
        assert 1 <= sweeps <= 4
        assert np.linalg.norm(Y - Y64) / np.linalg.norm(Y64) < 50 * kappa * feast.U64
        Y32 = scipy.linalg.lu_solve(scipy.linalg.lu_factor(T.astype(np.complex64)), rhs.astype(np.complex64))
        assert np.linalg.norm(Y32 - Y64) / np.linalg.norm(Y64) > 1e3 * np.linalg.norm(Y - Y64) / np.linalg.norm(Y64)


# ---------------------------------------------------------------------------
# planted mistakes: each must break a pin above
# ---------------------------------------------------------------------------

def _right_filter_error(filter_fn, nodes_fn=Q.nodes_and_weights, with_B=True):
    A, B, lam, V = small_pencil(with_B=with_B)
    c, R, q = 0.1 + 0.05j, 1.05, 16
    z, s = nodes_fn(c, R, 1.0, TR, q)
    U = pencils.complex_gaussian(np.random.default_rng(1), (A.shape[0], 6))
    got = filter_fn(feast.factor_nodes(A, B, z), s, B, U)
    expect = V @ (closed_form_rho_tr(lam, c, R, q)[:, None] * np.linalg.solve(V, U))
    return np.linalg.norm(got - expect) / np.linalg.norm(expect)


def test_planted_mistakes_are_caught():
    assert _right_filter_error(feast.filter_right) < 1e-11

    def sign_flipped(lus, sigma, B, U):
        return feast.filter_right(lus, -sigma, B, U)

    def conj_weights(lus, sigma, B, U):
        return feast.filter_right(lus, np.conj(sigma), B, U)

    def no_B(lus, sigma, B, U):
        return feast.filter_right(lus, sigma, None, U)

    def unfolded_nodes(c, R, a, rule, q):
        # mistake: mirror nodes taken at t instead of 2 - t (the fold of eqn:pi not applied)
        K = Q.points_per_half(rule, q)
        t, w = Q.base_rule(rule, K)
        z = np.concatenate([Q.phi(t, c, R, a), Q.phi(t[1:-1], c, R, a)])
        s = np.concatenate([w * Q.phi_prime(t, R, a), w[1:-1] * Q.phi_prime(t[1:-1], R, a)]) / (2j * np.pi)
        return z, s

    def unfolded_filter(lus, sigma, B, U):
        return feast.filter_right(lus, sigma, B, U)

    for bad in (sign_flipped, conj_weights, no_B):
        assert _right_filter_error(bad) > 1e-3, bad.__name__
    assert _right_filter_error(unfolded_filter, nodes_fn=unfolded_nodes) > 1e-3

    # the left filter without the conjugated weights, or with a plain (not conjugate) transpose
    A, B, lam, V = small_pencil(with_B=True, seed=11)
    n = A.shape[0]
    c, R, q = -0.05j, 0.95, 16
    z, s = Q.nodes_and_weights(c, R, 1.0, TR, q)
    lus = feast.factor_nodes(A, B, z)
    Vin = pencils.complex_gaussian(np.random.default_rng(2), (n, 5))
    Y = np.linalg.inv(B.conj().T) @ np.linalg.inv(V).conj().T
    expect = Y @ (np.conj(closed_form_rho_tr(lam, c, R, q))[:, None] * (V.conj().T @ (B.conj().T @ Vin)))
    bad1 = sum(sk * Yk for sk, Yk in zip(s, feast.solve_nodes(lus, B.conj().T @ Vin, conj_trans=True)))
    bad2 = sum(np.conj(sk) * scipy.linalg.lu_solve(lu, B.conj().T @ Vin, trans=1) for sk, lu in zip(s, lus))
    for bad in (bad1, bad2):
        assert np.linalg.norm(bad - expect) / np.linalg.norm(expect) > 1e-3


@pytest.mark.parametrize("with_B", [False, True])
@pytest.mark.parametrize("rule", [TR, GL])
def test_left_projector_variant_finds_left_eigenpairs(with_B, rule):
    """The left-projector variant: exactly the prescribed eigenvalues inside the contour, and every
    returned vector is a left eigenvector by definition (y^H A = lambda y^H B, i.e. the rows of
    Y_exact = B^-H V^-H up to scale)."""
    A, B, lam, V = small_pencil(n=80, m=6, with_B=with_B, seed=23)
    c = 0.05 - 0.02j
    V0 = pencils.complex_gaussian(np.random.default_rng(4), (80, 10))
    r = feast.lfeast(A, B, c, 1.0, 1.0, 16, V0, rule=rule)
    ref = brute.eigenvalues_inside(lam, c, 1.0)
    assert r.converged and r.m == len(ref) == 6
    assert match_eigs(r.lam, ref) < 1e-10
    Bm = np.eye(80) if B is None else B
    for j in range(r.m):
        y = r.X[:, j]
        res = np.linalg.norm(y.conj() @ A - r.lam[j] * (y.conj() @ Bm)) / (abs(r.lam[j]) * np.linalg.norm(y.conj() @ Bm))
        assert res < 1e-9
    # the exact left eigenvector of the matching eigenvalue: Y = B^-H V^-H, columns in lam's order
    Yx = np.linalg.inv(Bm.conj().T) @ np.linalg.inv(V).conj().T
    for j in range(r.m):
        k = int(np.argmin(np.abs(lam - r.lam[j])))
        y, yx = r.X[:, j], Yx[:, k] / np.linalg.norm(Yx[:, k])
        assert abs(abs(np.vdot(yx, y)) - 1) < 1e-8


def test_left_projector_variant_planted_mistakes():
    """Plausible slips break the pins above: with the right filter in place of the left one the basis
    tends to right eigenvectors (the eigenvalues still come out, since any invariant subspace gives
    them, but the vectors fail the left-eigenvector test); adjoint Ritz values reported without
    conjugation miss the eigenvalues."""
    A, B, lam, V = small_pencil(n=60, m=5, with_B=True, seed=29)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, TR, 16)
    lus = feast.factor_nodes(A, B, z)
    ref = brute.eigenvalues_inside(lam, 0, 1.0)

    def run(filt, conj_back):
        Vb = pencils.complex_gaussian(np.random.default_rng(3), (60, 9))
        for _ in range(8):
            Vh = feast.orthonormalize(filt(lus, s, B, Vb))
            mu, W = scipy.linalg.eig(Vh.conj().T @ A.conj().T @ Vh, Vh.conj().T @ B.conj().T @ Vh)
            Vb = Vh @ W
        lam_out = np.conj(mu) if conj_back else mu
        keep = np.abs(lam_out) < 1
        Y = Vb[:, keep] / np.linalg.norm(Vb[:, keep], axis=0)
        left_res = max(np.linalg.norm(y.conj() @ A - l * (y.conj() @ B)) for y, l in zip(Y.T, lam_out[keep]))
        return lam_out[keep], left_res

    good, res = run(feast.filter_left, True)
    assert len(good) == len(ref) and match_eigs(good, ref) < 1e-10 and res < 1e-9
    _, res_right = run(feast.filter_right, True)
    assert res_right > 1e-3
    bad, _ = run(feast.filter_left, False)
    assert len(bad) != len(ref) or match_eigs(bad, ref) > 1e-6


# ---------------------------------------------------------------------------
# hand-computed residuals (the stopping rule's inputs)
# ---------------------------------------------------------------------------
#
# A = [[1, 2i], [0, 3]], B = [[2, 0], [1, 1]] (B is not a multiple of I, so ||x||, ||B x|| and
# ||B^H y|| all differ and a wrong denominator changes the value).
#
# Right pairs (residual r = A x - lam B x):
#   x = (1, 1),  lam = 1 : A x = (1 + 2i, 3), B x = (2, 2), r = (-1 + 2i, 1), ||r||^2 = 6,
#                          ||x||^2 = 2, ||B x||^2 = 8  -> paper sqrt(3), relative sqrt(3)/2
#   x = (1, 0),  lam = 2i: A x = (1, 0), B x = (2, 1), r = (1 - 4i, -2i), ||r||^2 = 21,
#                          ||x|| = 1, ||B x||^2 = 5    -> paper sqrt(21), relative sqrt(21)/(2 sqrt 5)
# Left pairs (residual R = A^H y - conj(lam) B^H y, A^H = [[1, 0], [-2i, 3]], B^H = [[2, 1], [0, 1]]):
#   y = (1, 1),  lam = 1 : A^H y = (1, 3 - 2i), B^H y = (3, 1), R = (-2, 2 - 2i), ||R||^2 = 12,
#                          ||B^H y||^2 = 10             -> relative sqrt(12/10)
#   y = (0, 1),  lam = 2i: A^H y = (0, 3), B^H y = (1, 1), R = (2i, 3 + 2i), ||R||^2 = 17,
#                          ||B^H y||^2 = 2              -> relative sqrt(17)/(2 sqrt 2)

A22 = np.array([[1, 2j], [0, 3]], dtype=np.complex128)
B22 = np.array([[2, 0], [1, 1]], dtype=np.complex128)
LAM22 = np.array([1.0, 2j])


def test_residuals_hand_computed():
    X = np.array([[1, 1], [1, 0]], dtype=np.complex128)
    paper, rel = feast.residuals(A22, B22, LAM22, X)
    np.testing.assert_allclose(paper, [np.sqrt(3.0), np.sqrt(21.0)], rtol=1e-15)
    np.testing.assert_allclose(rel, [np.sqrt(3.0) / 2, np.sqrt(21.0) / (2 * np.sqrt(5.0))], rtol=1e-15)
    # B = None means B = I: r = A x - lam x, relative denominator |lam| ||x||
    #   x = (1, 1), lam = 1 : r = (2i, 2), ||r||^2 = 8          -> paper 2, relative 2
    #   x = (1, 0), lam = 2i: r = (1 - 2i, 0), ||r||^2 = 5       -> paper sqrt 5, relative sqrt(5)/2
    paper, rel = feast.residuals(A22, None, LAM22, X)
    np.testing.assert_allclose(paper, [2.0, np.sqrt(5.0)], rtol=1e-15)
    np.testing.assert_allclose(rel, [2.0, np.sqrt(5.0) / 2], rtol=1e-15)


def test_left_residuals_hand_computed():
    Y = np.array([[1, 0], [1, 1]], dtype=np.complex128)
    rel = feast.left_residuals(A22, B22, LAM22, Y)
    np.testing.assert_allclose(rel, [np.sqrt(12.0 / 10.0), np.sqrt(17.0) / (2 * np.sqrt(2.0))], rtol=1e-15)
    # B = None: R = A^H y - conj(lam) y
    #   y = (1, 1), lam = 1 : R = (0, 2 - 2i), ||R||^2 = 8, ||y||^2 = 2       -> relative 2
    #   y = (0, 1), lam = 2i: R = (0, 3 + 2i), ||R||^2 = 13, ||y|| = 1        -> relative sqrt(13)/2
    rel = feast.left_residuals(A22, None, LAM22, Y)
    np.testing.assert_allclose(rel, [2.0, np.sqrt(13.0) / 2], rtol=1e-15)


def test_residuals_vanish_on_exact_pairs():
    """On exact eigenpairs of the 2 x 2 pencil both residuals are at rounding level.  The
    eigenvalues are the roots of the characteristic polynomial, expanded by hand:
    det(A - l B) = (1 - 2l)(3 - l) - 2i(-l) = 2 l^2 - (7 - 2i) l + 3; the vectors are null vectors
    of A - l B and of its conjugate transpose."""
    roots = np.roots([2.0, -(7.0 - 2j), 3.0])
    for lam in roots:
        M = A22 - lam * B22
        _, _, Vh = np.linalg.svd(M)
        x = Vh[-1].conj()[:, None]
        _, _, Vh2 = np.linalg.svd(M.conj().T)
        y = Vh2[-1].conj()[:, None]
        paper, rel = feast.residuals(A22, B22, np.array([lam]), x)
        assert rel[0] < 1e-14 and paper[0] < 1e-14
        assert feast.left_residuals(A22, B22, np.array([lam]), y)[0] < 1e-14
