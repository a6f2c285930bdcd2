"""The shifted-residual form of the filter (feast_filter_shifted), which every FP32 and FP16
iteration after the first applies, against the oracle's plain FP64 filter.

For a block U and shifts l_j the library computes U rho(L) + sum_k sigma_k T_k^-1 (E D_k) with the
FP64 residual block E = A U - B U L and D_k = diag(1/(z_k - l_j)); in exact arithmetic this is
rho(M) U = sum_k sigma_k T_k^-1 B U (eqn:Rasp), which oracle.feast.filter_right computes in FP64
(and its left twin, eqn:quadf_surMconj).  The low-precision solves only see E D_k, so the
difference to the FP64 filter is bounded by the solves' relative error kappa(T_k) u_low times
sum_k |sigma_k| ||E D_k||, not by kappa u_low ||Q||: near eigenpairs (E small) the shifted form
must beat a plain FP32 filter by the factor ||E|| / ||B U||, which the tests check element by
element.
"""
import numpy as np
import pytest
import scipy.linalg

import pencils
from oracle import feast
from oracle import quadrature as Q
from tests.gpu_common import device, random_pencil

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
U16 = 2.0 ** -11


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


def expected_bound(A, B, z, s, U, lam, side, u_low, kappa):
    """kappa u_low sum_k |sigma_k| ||E D_k||_F: the shifted form's error budget, E in FP64."""
    n = A.shape[0]
    Bm = np.eye(n) if B is None else B
    if side == 0:
        E = A @ U - (Bm @ U) * lam[None, :]
        D = [1.0 / (zk - lam) for zk in z]
    else:
        E = A.conj().T @ U - (Bm.conj().T @ U) * np.conj(lam)[None, :]
        D = [np.conj(1.0 / (zk - lam)) for zk in z]
    return kappa * u_low * sum(abs(sk) * np.linalg.norm(E * dk[None, :]) for sk, dk in zip(s, D))


def near_pairs(A, B, lam_all, idx, eps, rng, side=0):
    """Exact right (side 0) or left (side 1: A^H y = conj(l) B^H y) eigenvectors of the selected
    eigenvalues, perturbed by eps (relative), with the eigenvalues perturbed by eps as shifts: a
    block like the iteration's Ritz pairs before convergence."""
    n = A.shape[0]
    Bm = np.eye(n) if B is None else B
    if side == 0:
        w, V = scipy.linalg.eig(A, Bm)
    else:
        w, V = scipy.linalg.eig(A.conj().T, Bm.conj().T)
        w = np.conj(w)
    cols = [int(np.argmin(np.abs(w - lam_all[i]))) for i in idx]
    U = V[:, cols]
    U = U / np.linalg.norm(U, axis=0)[None, :]
    U = U + eps * pencils.complex_gaussian(rng, U.shape) / np.sqrt(n)
    lam = w[cols] * (1 + eps * (rng.standard_normal(len(cols)) + 1j * rng.standard_normal(len(cols))))
    return np.asfortranarray(U), lam


@pytest.mark.parametrize("n,with_B", [(300, True), (257, False), (520, True)])
@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_shifted_filter_near_eigenpairs(n, with_B, side, prec):
    A, B, lam_all = random_pencil(n, seed=5 * n + side, with_B=with_B, m=6, cond=10.0)
    q, m0 = 16, 12
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", q)
    rng = np.random.default_rng(n + 17 * side)
    inside = np.flatnonzero(np.abs(lam_all) < 1.0)
    outside = np.flatnonzero(np.abs(lam_all) >= 1.0)[: m0 - len(inside)]
    U, lam = near_pairs(A, B, lam_all, list(inside) + list(outside), 1e-6, rng, side)
    lus = feast.factor_nodes(A, B, z)
    ref = feast.filter_right(lus, s, B, U) if side == 0 else feast.filter_left(lus, s, B, U)
    kappa = max(np.linalg.cond(feast.node_matrix(A, B, zk)) for zk in z)
    u_low = U32 if prec == "fp32" else U16
    with fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, precision=prec, pivoting="partial") as F:
        got = F.filter_shifted(upload(U), lam, side).cpu().numpy()
        plain = F.filter(upload(U), side).cpu().numpy() if prec == "fp32" else None
    bound = expected_bound(A, B, z, s, U, lam, side, u_low, kappa)
    err = np.abs(got - ref)
    # element by element: every entry within the budget of the solves plus FP64 rounding
    assert err.max() <= 10 * bound + 1e-12 * np.abs(ref).max(), (err.max(), bound)
    # the budget itself is far below a plain low-precision filter's error level kappa u_low ||Q||
    assert bound < 1e-3 * kappa * u_low * np.linalg.norm(ref)
    if plain is not None:
        # feast_filter refines its FP32 solves to FP64 accuracy: both forms agree with the oracle
        assert np.abs(plain - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("side", [0, 1])
def test_shifted_filter_arbitrary_shifts(side):
    """Random U and shifts off the nodes: E is as large as B U, the identity still holds and the
    error stays within kappa u32 sum_k |sigma_k| ||E D_k||."""
    n, q, m0 = 200, 16, 8
    A, B, lam_all = random_pencil(n, seed=31 + side, with_B=True, cond=5.0)
    z, s = Q.nodes_and_weights(0.1 + 0.05j, 1.1, 1.0, "trapezoid", q)
    rng = np.random.default_rng(9 + side)
    U = np.asfortranarray(pencils.complex_gaussian(rng, (n, m0)))
    lam = 0.6 * (rng.standard_normal(m0) + 1j * rng.standard_normal(m0))
    lus = feast.factor_nodes(A, B, z)
    ref = feast.filter_right(lus, s, B, U) if side == 0 else feast.filter_left(lus, s, B, U)
    kappa = max(np.linalg.cond(feast.node_matrix(A, B, zk)) for zk in z)
    with fm().Feast(upload(A), upload(B), 0.1 + 0.05j, 1.1, 1.0, q, m0, precision="fp32") as F:
        got = F.filter_shifted(upload(U), lam, side).cpu().numpy()
    bound = expected_bound(A, B, z, s, U, lam, side, U32, kappa)
    assert np.abs(got - ref).max() <= 10 * bound + 1e-12 * np.abs(ref).max()


def test_shifted_filter_fp64_and_conjugate_nodes():
    """FP64 factorisations: the shifted form equals the plain filter to FP64 rounding; with
    shared conjugate nodes (a real pencil) the mirror terms are added as in the iteration."""
    n, q, m0 = 300, 16, 10
    rng = np.random.default_rng(4)
    A, B, _ = pencils.real_pencil(rng, n, 3, 2)     # real, 8 eigenvalues in |z| < 0.8, rest beyond 1.5
    A, B = np.asfortranarray(A, dtype=np.complex128), np.asfortranarray(B, dtype=np.complex128)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "gauss-legendre", q)
    U = np.asfortranarray(pencils.complex_gaussian(rng, (n, m0)))
    lam = 0.3 * (rng.standard_normal(m0) + 1j * rng.standard_normal(m0))
    ref = feast.filter_right(feast.factor_nodes(A, B, z), s, B, U)
    for prec, conj, tol in (("fp64", "none", 1e-11), ("fp64", "real", 1e-11), ("fp32", "real", None)):
        with fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, rule="gauss-legendre", precision=prec,
                        conj_nodes=conj) as F:
            got = F.filter_shifted(upload(U), lam, 0).cpu().numpy()
        if tol is None:
            kappa = max(np.linalg.cond(feast.node_matrix(A, B, zk)) for zk in z)
            bound = 10 * expected_bound(A, B, z, s, U, lam, 0, U32, kappa) + 1e-12 * np.abs(ref).max()
        else:
            bound = tol * np.abs(ref).max()
        assert np.abs(got - ref).max() <= bound, (prec, conj, np.abs(got - ref).max(), bound)


def test_shifted_filter_rejects_bad_arguments():
    A, B, _ = random_pencil(64, seed=2, with_B=False)
    z, _ = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", 8)
    with fm().Feast(upload(A), None, 0j, 1.0, 1.0, 8, 4, precision="fp32") as F:
        U = upload(np.ones((64, 4), dtype=np.complex128))
        with pytest.raises(fm().FeastError):
            F.filter_shifted(U, [z[0], 0.1, 0.2, 0.3])      # a shift on a node
        with pytest.raises(ValueError):
            F.filter_shifted(U, [0.1, 0.2])


def test_iteration_with_classic_refinement_sweeps():
    """feast_iterate with ir_tol > 0 replaces the shifted-residual correction by classic FP64
    refinement sweeps of every node solve (R_k = B U - T_k Y_k in FP64, low-precision correction)
    in every filter: on the 200 x 200 workload in FP32 it reaches the prescribed eigenvalues to
    1e-10 like the default, and reports the sweeps it ran."""
    from oracle import brute
    from tests.gpu_common import match_eigs
    P = pencils.c0()
    A = upload(P.A)
    U0 = upload(pencils.start_block(0, P.n, P.m0))
    ref = brute.eigenvalues_inside(P.lam, P.center, P.radius)
    with fm().Feast(A, None, P.center, P.radius, 1.0, P.q, P.m0, precision="fp32", ir_tol=1e-12) as F:
        r = F.iterate(U0)
    assert r.converged and len(r.lam) == len(ref), r.history
    assert match_eigs(r.lam, ref) < 1e-10 and np.all(r.resid <= 1e-10)
    assert r.ir_sweeps > 0
    with fm().Feast(A, None, P.center, P.radius, 1.0, P.q, P.m0, precision="fp32") as F:
        d = F.iterate(U0)
    assert d.converged and d.ir_sweeps == 0 and match_eigs(d.lam, ref) < 1e-10
