"""The left-projector variant (variant "L": Section 4's one-projector algorithm with the left
projector) on the device, against the oracle's iteration and the definition of left eigenvectors."""
import numpy as np
import pytest

import pencils
from oracle import brute, feast
from tests.gpu_common import device, match_eigs, random_pencil

pytestmark = pytest.mark.gpu


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


def check_left_pairs(res, A, B, ref, tol=1e-10):
    assert res.converged and len(res.lam) == len(ref), (len(res.lam), len(ref), res.history)
    assert match_eigs(res.lam, ref) < tol
    assert np.all(res.resid <= 1e-10)
    Y = res.X.cpu().numpy()
    Bm = np.eye(A.shape[0]) if B is None else B
    for j in range(len(res.lam)):
        y = Y[:, j]
        r = np.linalg.norm(y.conj() @ A - res.lam[j] * (y.conj() @ Bm)) / (abs(res.lam[j]) * np.linalg.norm(y.conj() @ Bm))
        assert r < 1e-9, (j, r)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("with_B", [False, True])
def test_left_variant_matches_oracle(prec, with_B):
    n = 300
    A, B, lam = random_pencil(n, seed=41, with_B=with_B, m=9)
    c = 0.03 - 0.02j
    ref = brute.eigenvalues_inside(lam, c, 1.0)
    V0 = pencils.complex_gaussian(np.random.default_rng(2), (n, 16))
    F = fm().Feast(upload(A), upload(B), c, 1.0, 1.0, 16, 16, precision=prec, variant="L")
    r = F.iterate(upload(V0))
    check_left_pairs(r, A, B, ref)
    orc = feast.lfeast(A, B, c, 1.0, 1.0, 16, V0)
    assert match_eigs(r.lam, orc.lam) < 1e-10
    if prec != "fp16":
        # (FP16 factors filter less sharply in the first iterations: more iterations, same result)
        assert abs(r.iterations - orc.iters) <= 1
    F.close()


def test_left_variant_c0_and_full_size_sample():
    """The 200 x 200 workload, and its left vectors against the exact ones Y = V^-H."""
    P = pencils.c0()
    V0 = pencils.start_block(0, P.n, P.m0)
    F = fm().Feast(upload(P.A), None, P.center, P.radius, 1.0, P.q, P.m0, variant="L", precision="fp32")
    r = F.iterate(upload(V0))
    check_left_pairs(r, P.A, None, brute.eigenvalues_inside(P.lam, P.center, P.radius))
    F.close()


def test_left_variant_glued_contour_and_shared_conjugate_nodes():
    """Left projector on a real pencil with shared conjugate nodes (13 of 24 factored)."""
    n = 300
    A, B, lam = pencils.real_pencil(np.random.default_rng(21), n, 4, 2)
    ref = brute.eigenvalues_inside(lam, 0j, 1.0)
    V0 = pencils.complex_gaussian(np.random.default_rng(4), (n, 16))
    for prec in ("fp64", "fp32"):
        F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, 24, 16, variant="L", precision=prec, conj_nodes="real")
        check_left_pairs(F.iterate(upload(V0)), A, B, ref)
        F.close()


def test_left_variant_in_a_batch():
    P = [pencils.c2_pencil(j, 200 + 60 * j, 6 + j) for j in range(3)]
    dev = [(upload(p.A), upload(p.B)) for p in P]
    batch = fm().FeastBatch(dev, (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16, variant="L")
    V0 = [upload(pencils.start_block(2, p.n, p.m0, salt=10 ** 6 + j)) for j, p in enumerate(P)]
    res, rcs = batch.iterate(V0)
    assert list(rcs) == [0, 0, 0]
    for r, p in zip(res, P):
        check_left_pairs(r, p.A, p.B, brute.eigenvalues_inside(p.lam, 0j, 1.0))
    batch.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_left_variant_on_a_contour_not_symmetric_about_the_real_axis(prec):
    """The triangle 0, 2, 1 + 1.5i lies above the real axis, so the candidates' inside test must use
    lambda, not the adjoint Ritz value conj(lambda): with the wrong one no candidate would be found."""
    from tests.glued_shapes import SHAPES, glued_spectrum
    pieces, _, member = SHAPES["triangle"]
    n = 300
    lam0 = glued_spectrum("triangle", n, 10, seed=8)
    A, B, lam = random_pencil(n, seed=3, with_B=True, spectrum=lam0)
    ref = lam0[member(lam0)]
    V0 = pencils.complex_gaussian(np.random.default_rng(5), (n, 18))
    F = fm().Feast(upload(A), upload(B), q=24, m0=18, precision=prec, variant="L", max_iter=40, pieces=pieces)
    check_left_pairs(F.iterate(upload(V0)), A, B, ref)
    F.close()
