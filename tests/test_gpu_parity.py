"""Parity of the HIP path with the CPU oracle, element by element, through the C-ABI.

Tolerances (FP64 path): a backward-stable LU solve has forward error <= c n kappa(T) u; the tests
use 50 kappa u with kappa measured by the oracle (NumPy cond).  FP32 + FP64 refinement: the
refined solve converges to the FP64 solution, tolerance 200 kappa u64.  Eigenvalues: 1e-10
relative (spec bound for the FP64 path) after optimal assignment, equal counts.
"""
import numpy as np
import pytest
import scipy.linalg

import pencils
from oracle import brute, feast
from oracle import quadrature as Q
from tests.gpu_common import device, golden_spectrum, match_eigs, random_pencil, rel_err

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


def host(t):
    return t.cpu().numpy()


# ---------------------------------------------------------------------------
# a2 + a3 + a5: per-node factor and solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 65, 129, 200, 257])
@pytest.mark.parametrize("with_B", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_node_solve_matches_oracle(n, with_B, prec):
    A, B, lam = random_pencil(n, seed=n, with_B=with_B)
    q, m0 = 8, min(n, 7)
    c, R = 0.05 + 0.02j, 1.0
    F = fm().Feast(upload(A), upload(B), c, R, 1.0, q, m0, precision=prec)
    z, s = Q.nodes_and_weights(c, R, 1.0, "trapezoid", q)
    rhs = pencils.complex_gaussian(np.random.default_rng(n + 1), (n, m0))
    rd = upload(rhs)
    for k in (0, 3, q - 1):
        T = feast.node_matrix(A, B, z[k])
        kappa = np.linalg.cond(T)
        for side in (0, 1):
            got = host(F.node_solve(k, rd, side))
            ref = scipy.linalg.lu_solve(scipy.linalg.lu_factor(T), rhs, trans=2 if side else 0)
            tol = (50 if prec == "fp64" else 200) * kappa * U64 * max(1, np.sqrt(n) / 4)
            assert rel_err(got, ref) < tol, (k, side, rel_err(got, ref), tol)
    F.close()


def test_singular_node_is_reported():
    """An eigenvalue placed exactly on node 0 (z_0 = c + R = 1 for the unit circle) makes that node
    matrix exactly singular: setup must report FEAST_ESINGULAR + 0."""
    n = 32
    d = np.linspace(1.5, 3.0, n).astype(np.complex128)
    d[5] = 1.0
    A = np.asfortranarray(np.diag(d))
    with pytest.raises(fm().FeastError) as e:
        fm().Feast(upload(A), None, 0j, 1.0, 1.0, 16, 4)
    assert e.value.code == fm().binding.FEAST_ESINGULAR + 0


# ---------------------------------------------------------------------------
# a4 - a7: the filter
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,q,m0", [(64, 8, 8), (200, 16, 16), (321, 16, 5), (513, 24, 33)])
@pytest.mark.parametrize("with_B", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("pivoting", ["tournament", "partial"])
def test_filter_matches_oracle(n, q, m0, with_B, prec, pivoting):
    A, B, lam = random_pencil(n, seed=3 * n + q, with_B=with_B)
    c, R = 0.02 - 0.01j, 1.0
    F = fm().Feast(upload(A), upload(B), c, R, 1.0, q, m0, precision=prec, pivoting=pivoting)
    z, s = Q.nodes_and_weights(c, R, 1.0, "trapezoid", q)
    lus = feast.factor_nodes(A, B, z)
    U = pencils.complex_gaussian(np.random.default_rng(n), (n, m0))
    kappa = max(np.linalg.cond(feast.node_matrix(A, B, zk)) for zk in z)
    tol = (50 if prec == "fp64" else 200) * kappa * U64 * max(1, np.sqrt(n) / 4)
    for side in (0, 1):
        got = host(F.filter(upload(U), side))
        ref = (feast.filter_right if side == 0 else feast.filter_left)(lus, s, B, U)
        assert rel_err(got, ref) < tol, (side, rel_err(got, ref), tol)
    F.close()


def test_filter_closed_form_prescribed_spectrum():
    """eqn:quadf_surM on the device: Q = V rho(L) V^-1 U with the closed-form trapezoid filter."""
    P = pencils.c0()
    F = fm().Feast(upload(P.A), None, 0j, 1.0, 1.0, 16, 16)
    U = pencils.start_block(0, P.n, 16)
    got = host(F.filter(upload(U)))
    g = np.random.default_rng([pencils.base_seed(0), 0])
    lam = pencils.prescribed_spectrum(g, P.n, 10)
    V = pencils.clipped_gaussian_basis(g, P.n, 1e3)
    expect = V @ ((1 / (1 - lam ** 16))[:, None] * np.linalg.solve(V, U))
    assert rel_err(got, expect) < 1e-10
    F.close()


def test_filter_ragged_column_counts():
    A, B, lam = random_pencil(150, seed=5, with_B=True)
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, 8, 20)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", 8)
    lus = feast.factor_nodes(A, B, z)
    for k in (1, 3, 16, 17, 20):
        U = pencils.complex_gaussian(np.random.default_rng(k), (150, k))
        assert rel_err(host(F.filter(upload(U))), feast.filter_right(lus, s, B, U)) < 1e-11
    F.close()


# ---------------------------------------------------------------------------
# a8: R-FEAST / Bi-FEAST end to end
# ---------------------------------------------------------------------------

def check_eigenpairs(res, A, B, ref_lam, tol=1e-10):
    assert res.converged
    assert len(res.lam) == len(ref_lam)
    assert match_eigs(res.lam, ref_lam) < tol
    assert np.all(res.resid <= 1e-10)
    X = host(res.X)
    Bm = np.eye(A.shape[0]) if B is None else B
    for j in range(len(res.lam)):
        x = X[:, j]
        r = np.linalg.norm(A @ x - res.lam[j] * (Bm @ x)) / (abs(res.lam[j]) * np.linalg.norm(Bm @ x))
        assert r < 1e-9
        assert abs(np.linalg.norm(x) - 1) < 1e-10


@pytest.mark.parametrize("variant", ["R", "Bi"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_iterate_c0(variant, prec):
    P = pencils.c0()
    U0 = pencils.start_block(0, P.n, P.m0)
    F = fm().Feast(upload(P.A), None, P.center, P.radius, 1.0, P.q, P.m0, precision=prec, variant=variant)
    res = F.iterate(upload(U0))
    ref = brute.eigenvalues_inside(P.lam, P.center, P.radius)
    check_eigenpairs(res, P.A, None, ref)
    orc = (feast.rfeast if variant == "R" else feast.bifeast)(P.A, None, 0j, 1.0, 1.0, 16, U0)
    assert match_eigs(res.lam, orc.lam) < 1e-10
    assert abs(res.iterations - orc.iters) <= 1
    if variant == "Bi":
        Y = host(res.Y)
        X = host(res.X)
        G = Y.conj().T @ X
        assert np.allclose(G, np.diag(np.diag(G)), atol=1e-8)
    F.close()


@pytest.mark.parametrize("variant", ["R", "Bi"])
def test_iterate_generalized(variant):
    A, B, lam = random_pencil(300, seed=77, with_B=True, m=9)
    U0 = pencils.complex_gaussian(np.random.default_rng(1), (300, 14))
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, 16, 14, variant=variant)
    res = F.iterate(upload(U0))
    check_eigenpairs(res, A, B, brute.eigenvalues_inside(lam, 0, 1.0))
    F.close()


@pytest.mark.parametrize("variant", ["R", "Bi"])
@pytest.mark.parametrize("m0", [14, 80, 128, 136])
def test_iterate_device_and_host_orthonormalisation(variant, m0):
    """The shifted Cholesky-QR passes with the Gram matrices factored on the device (default; the
    packed factor of an order up to 128 lives in LDS, above in global memory) and on the host reach
    the same eigenpairs: equal counts, eigenvalues within 1e-10 relative of each other and of the
    brute-force spectrum, iteration counts within one."""
    A, B, lam = random_pencil(300, seed=78, with_B=True, m=9)
    U0 = pencils.complex_gaussian(np.random.default_rng(3), (300, m0))
    out = {}
    for host_ortho in (False, True):
        F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, 16, m0, variant=variant, host_ortho=host_ortho)
        res = F.iterate(upload(U0))
        check_eigenpairs(res, A, B, brute.eigenvalues_inside(lam, 0, 1.0))
        out[host_ortho] = res
        F.close()
    assert len(out[False].lam) == len(out[True].lam) == 9
    assert match_eigs(out[False].lam, out[True].lam) < 1e-10
    assert abs(out[False].iterations - out[True].iterations) <= 1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("host_ortho", [False, True])
def test_iterate_zero_start_block_reports_reduced_failure(prec, host_ortho):
    """A zero start block filters to a zero block whose Gram matrix has zero trace: the shifted
    Cholesky-QR cannot factor it, on the device (its failure flag) or on the host, and the iteration
    stops with FEAST_EREDUCED instead of producing vectors."""
    A, B, lam = random_pencil(150, seed=12, with_B=True, m=5)
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, 16, 8, precision=prec, host_ortho=host_ortho)
    with pytest.raises(fm().FeastError) as err:
        F.iterate(upload(np.zeros((150, 8), dtype=np.complex128)))
    assert err.value.code == fm().binding.FEAST_EREDUCED
    # the context stays usable
    res = F.iterate(upload(pencils.complex_gaussian(np.random.default_rng(4), (150, 8))))
    check_eigenpairs(res, A, B, brute.eigenvalues_inside(lam, 0, 1.0))
    F.close()


def test_iterate_empty_contour():
    """No eigenvalue inside: the iteration stops with m = 0."""
    A, B, lam = random_pencil(120, seed=4, with_B=False, m=0)
    U0 = pencils.complex_gaussian(np.random.default_rng(2), (120, 8))
    F = fm().Feast(upload(A), None, 0j, 1.0, 1.0, 16, 8)
    res = F.iterate(upload(U0))
    assert res.converged and len(res.lam) == 0
    F.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_iterate_full_size_complex_symmetric(prec):
    """n = 4096 complex-symmetric generalized pencil (q = 24, m0 = 64), radius R* from the golden
    spectrum: the candidates are exactly the m eigenvalues the oracle finds inside (shift-invert
    Arnoldi reference, stored with the golden data), to 1e-10 relative.  In the FP16 mode (scaled
    FP16 trailing updates + FP64 correction) the node systems of this pencil are too ill-conditioned
    for FP16 factors, so the iteration stalls and replaces them by FP32 ones (recorded in the result)
    before it converges."""
    g = golden_spectrum("c1")
    P = pencils.c1(radius=g["radius"])
    U0 = pencils.start_block(1, P.n, P.m0)
    F = fm().Feast(upload(P.A), upload(P.B), P.center, P.radius, 1.0, P.q, P.m0, precision=prec)
    res = F.iterate(upload(U0))
    ref = g["nearest"][: g["m"]]
    assert res.converged
    assert res.escalated == (prec == "fp16")
    assert len(res.lam) == g["m"]
    assert match_eigs(res.lam, ref) < 1e-10
    assert np.all(res.resid <= 1e-10)
    # sampled eigenvectors checked on the host
    X = host(res.X)
    for j in (0, len(res.lam) // 2, len(res.lam) - 1):
        x = X[:, j]
        r = np.linalg.norm(P.A @ x - res.lam[j] * (P.B @ x)) / (abs(res.lam[j]) * np.linalg.norm(P.B @ x))
        assert r < 1e-9
    F.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_bifeast_full_size_n8192(prec):
    """n = 8192 complex-symmetric generalized pencil, q = 32, m0 = 128, Bi-FEAST (right and left
    solves from one factorisation per node), radius R* from the golden spectrum: the candidates are
    the m eigenvalues inside (oracle shift-invert reference) to 1e-10 relative; sampled right and left
    eigenvectors are checked on the host.  The FP16 mode (scaled FP16 trailing updates + FP64
    correction) reaches the same eigenpairs after replacing its factors by FP32 ones (recorded)."""
    g = golden_spectrum("c3")
    P = pencils.c3(radius=g["radius"])
    U0 = pencils.start_block(3, P.n, P.m0)
    F = fm().Feast(upload(P.A), upload(P.B), P.center, P.radius, 1.0, P.q, P.m0, precision=prec, variant="Bi")
    res = F.iterate(upload(U0))
    ref = g["nearest"][: g["m"]]
    assert res.converged, res.history
    assert res.escalated == (prec == "fp16")
    assert len(res.lam) == g["m"]
    assert match_eigs(res.lam, ref) < 1e-10
    assert np.all(res.resid <= 1e-10)
    X = host(res.X)
    Y = host(res.Y)
    for j in (0, len(res.lam) // 2, len(res.lam) - 1):
        lam = res.lam[j]
        x, y = X[:, j], Y[:, j]
        r = np.linalg.norm(P.A @ x - lam * (P.B @ x)) / (abs(lam) * np.linalg.norm(P.B @ x))
        rl = np.linalg.norm(P.A.conj().T @ y - np.conj(lam) * (P.B.conj().T @ y)) / (
            abs(lam) * np.linalg.norm(P.B.conj().T @ y))
        assert r < 1e-9 and rl < 1e-8, (j, r, rl)
    F.close()
