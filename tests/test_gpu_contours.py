"""Other domains and rules (Section 3): Gauss-Legendre nodes, ellipses (aspect a != 1), shifted
circles, and glued contours (Section 5.4: triangle, square, semicircle, and two non-convex shapes),
on the device against the oracle's filter and iteration and the brute-force spectrum."""
import numpy as np
import pytest

import pencils
from oracle import brute, feast
from oracle import quadrature as Q
from tests.glued_shapes import SHAPES, glued_spectrum
from tests.gpu_common import device, match_eigs, random_pencil, rel_err

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


@pytest.mark.parametrize("rule,q", [("gauss-legendre", 8), ("gauss-legendre", 16), ("trapezoid", 12)])
@pytest.mark.parametrize("c,R,a", [(0j, 1.0, 0.6), (0.2 - 0.1j, 0.9, 1.0), (-0.1 + 0.05j, 1.1, 1.7)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_filter_other_contours_match_oracle(rule, q, c, R, a, prec):
    n, m0 = 257, 9
    A, B, lam = random_pencil(n, seed=q + 7, with_B=True)
    F = fm().Feast(upload(A), upload(B), c, R, a, q, m0, rule=rule, precision=prec)
    z, s = Q.nodes_and_weights(c, R, a, rule, q)
    lus = feast.factor_nodes(A, B, z)
    U = pencils.complex_gaussian(np.random.default_rng(q), (n, m0))
    kappa = max(np.linalg.cond(feast.node_matrix(A, B, zk)) for zk in z)
    tol = (50 if prec == "fp64" else 200) * kappa * U64 * 4
    for side in (0, 1):
        got = F.filter(upload(U), side).cpu().numpy()
        ref = (feast.filter_right if side == 0 else feast.filter_left)(lus, s, B, U)
        assert rel_err(got, ref) < tol, (side, rel_err(got, ref), tol)
    F.close()


@pytest.mark.parametrize("variant", ["R", "Bi"])
def test_iterate_ellipse_gauss_legendre(variant):
    """An ellipse with semi-axes 1 and 0.7 around the origin, 16 Gauss-Legendre nodes: the iteration
    finds exactly the prescribed eigenvalues inside the ellipse."""
    A, B, lam = random_pencil(300, seed=31, with_B=True, m=14)
    a = 0.7
    ref = brute.eigenvalues_inside(lam, 0j, 1.0, a)
    U0 = pencils.complex_gaussian(np.random.default_rng(5), (300, len(ref) + 8))
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, a, 16, len(ref) + 8, rule="gauss-legendre", variant=variant,
                   max_iter=40)
    r = F.iterate(upload(U0))
    assert r.converged and len(r.lam) == len(ref), (len(r.lam), len(ref), r.history)
    assert match_eigs(r.lam, ref) < 1e-10
    F.close()


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("rule", ["trapezoid", "gauss-legendre"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_filter_glued_contours_match_oracle(shape, rule, prec):
    """Eight rule points per piece; the right and left filters against the oracle's."""
    pieces = SHAPES[shape][0]
    n, m0, q = 257, 9, 8 * len(pieces)
    A, B, lam = random_pencil(n, seed=len(shape), with_B=True)
    F = fm().Feast(upload(A), upload(B), q=q, m0=m0, rule=rule, precision=prec, pieces=pieces)
    z, s = Q.glued_nodes_and_weights(pieces, rule, q)
    lus = feast.factor_nodes(A, B, z)
    U = pencils.complex_gaussian(np.random.default_rng(q), (n, m0))
    kappa = max(np.linalg.cond(feast.node_matrix(A, B, zk)) for zk in z)
    tol = (50 if prec == "fp64" else 200) * kappa * U64 * 4
    for side in (0, 1):
        got = F.filter(upload(U), side).cpu().numpy()
        ref = (feast.filter_right if side == 0 else feast.filter_left)(lus, s, B, U)
        assert rel_err(got, ref) < tol, (side, rel_err(got, ref), tol)
    F.close()


@pytest.mark.parametrize("shape,q,rule,variant", [
    ("triangle", 24, "trapezoid", "Bi"), ("square", 32, "trapezoid", "Bi"), ("semicircle", 16, "trapezoid", "Bi"),
    ("pacman", 48, "gauss-legendre", "R"), ("lshape", 48, "gauss-legendre", "R"), ("triangle", 24, "trapezoid", "R")])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_iterate_glued_contours(shape, q, rule, variant, prec):
    """The paper's domain-shape runs use Bi-FEAST with the trapezoid rule and 8 points per piece: the
    iteration finds exactly the prescribed eigenvalues inside the shape (candidate test: winding
    number), to 1e-10, in the oracle's iteration count (+-1)."""
    pieces, _, member = SHAPES[shape]
    n, m_in, m0 = 300, 10, 18
    lam0 = glued_spectrum(shape, n, m_in, seed=len(shape))
    A, B, lam = random_pencil(n, seed=3, with_B=True, spectrum=lam0)
    ref = lam0[member(lam0)]
    assert len(ref) == m_in
    U0 = pencils.complex_gaussian(np.random.default_rng(5), (n, m0))
    F = fm().Feast(upload(A), upload(B), q=q, m0=m0, rule=rule, variant=variant, precision=prec, max_iter=40,
                   pieces=pieces)
    r = F.iterate(upload(U0))
    assert r.converged and len(r.lam) == m_in, (len(r.lam), r.history)
    assert match_eigs(r.lam, ref) < 1e-10
    assert np.all(r.resid <= 1e-10)
    orc = (feast.rfeast if variant == "R" else feast.bifeast)(A, B, 0j, 1.0, 1.0, q, U0, rule=rule, max_iter=40,
                                                               pieces=pieces)
    assert abs(r.iterations - orc.iters) <= 1, (r.iterations, orc.iters)
    F.close()


def test_batch_mixes_glued_and_elliptic_contours():
    """One batch, one launch sequence: a triangle (glued, 8 trapezoid points per piece) and a circle
    share q = 24; each member finds its own enclosed eigenvalues."""
    pieces, _, member = SHAPES["triangle"]
    n = 200
    lam_t = glued_spectrum("triangle", n, 7, seed=11)
    A1, B1, _ = random_pencil(n, seed=12, with_B=True, spectrum=lam_t)
    A2, B2, lam_c = random_pencil(n, seed=13, with_B=False, m=6)
    dev = [(upload(A1), upload(B1)), (upload(A2), None)]
    batch = fm().FeastBatch(dev, [pieces, (0j, 1.0, 1.0)], m0=14, q=24)
    U0 = [upload(pencils.complex_gaussian(np.random.default_rng(j), (n, 14))) for j in range(2)]
    res, rcs = batch.iterate(U0)
    assert list(rcs) == [0, 0]
    assert res[0].converged and match_eigs(res[0].lam, lam_t[member(lam_t)]) < 1e-10
    assert res[1].converged and match_eigs(res[1].lam, brute.eigenvalues_inside(lam_c, 0j, 1.0)) < 1e-10
    batch.close()
