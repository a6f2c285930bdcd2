"""FP32 mode with the trailing updates on FP16 matrix cores and split operands (split_update): every
operand entry is carried as a high and a low FP16 part, so the factors keep about 22 significant
bits.  Checked against the FP64 solves of the oracle (the unrefined solves stay within a small factor
of the plain FP32 factors' error, far below the FP16 mode's), and end to end against the oracle's
eigenvalues."""
import numpy as np
import pytest
import scipy.linalg

import pencils
from oracle import brute, feast
from oracle import quadrature as Q
from tests.gpu_common import device, golden_spectrum, match_eigs, random_pencil, rel_err

pytestmark = pytest.mark.gpu
U22 = 2.0 ** -22


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


def host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("pivoting", ["tournament", "partial"])
@pytest.mark.parametrize("n", [65, 200, 257, 520, 1100])
def test_unrefined_split_solve_error(n, pivoting):
    """ir_max = 0 (plain solves with the factors): the split-update factors' error against the FP64
    solve is within 8x of the plain FP32 factors' (about 2^-22 against 2^-24 per operand) and at
    most 100 n^(1/2) kappa 2^-22, while the FP16-update factors' error is far above both; nodes 0
    and 5 of an 8-node circle (several update tiles and a ragged tail at n = 200, 520, 1100)."""
    A, B, lam = random_pencil(n, seed=n + 11, with_B=True, cond=3.0)
    q, m0 = 8, 6
    kw = dict(ir_max=0, pivoting=pivoting)
    Fs = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, precision="fp32", split_update=True, **kw)
    F32 = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, precision="fp32", **kw)
    F16 = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, precision="fp16", **kw)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", q)
    rhs = pencils.complex_gaussian(np.random.default_rng(n), (n, m0))
    rd = upload(rhs)
    for k in (0, 5):
        T = feast.node_matrix(A, B, z[k])
        exact = scipy.linalg.lu_solve(scipy.linalg.lu_factor(T), rhs)
        kappa = np.linalg.cond(T)
        e_s = rel_err(host(Fs.node_solve(k, rd)), exact)
        e_32 = rel_err(host(F32.node_solve(k, rd)), exact)
        e_16 = rel_err(host(F16.node_solve(k, rd)), exact)
        assert e_s <= 8 * e_32 + 1e-7, (k, e_s, e_32)
        assert e_s <= 100 * np.sqrt(n) * kappa * U22, (k, e_s, kappa)
        if n > 64:
            assert e_s * 20 < e_16, (k, e_s, e_16)
    for F in (Fs, F32, F16):
        F.close()


@pytest.mark.parametrize("n", [200, 520])
def test_refined_split_solve_reaches_fp64(n):
    A, B, lam = random_pencil(n, seed=n + 3, with_B=True)
    q, m0 = 8, 6
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, precision="fp32", split_update=True)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", q)
    rhs = pencils.complex_gaussian(np.random.default_rng(n + 1), (n, m0))
    for k in (1, 6):
        T = feast.node_matrix(A, B, z[k])
        exact = scipy.linalg.lu_solve(scipy.linalg.lu_factor(T), rhs)
        assert rel_err(host(F.node_solve(k, upload(rhs))), exact) < 200 * np.linalg.cond(T) * 2.0 ** -53
    F.close()


@pytest.mark.parametrize("variant", ["R", "Bi"])
def test_iterate_split_c0(variant):
    P = pencils.c0()
    U0 = pencils.start_block(0, P.n, P.m0)
    F = fm().Feast(upload(P.A), None, P.center, P.radius, 1.0, P.q, P.m0, precision="fp32", variant=variant,
                   split_update=True)
    res = F.iterate(upload(U0))
    ref = brute.eigenvalues_inside(P.lam, P.center, P.radius)
    assert res.converged and len(res.lam) == len(ref)
    assert match_eigs(res.lam, ref) < 1e-10
    orc = (feast.rfeast if variant == "R" else feast.bifeast)(P.A, None, 0j, 1.0, 1.0, 16, U0)
    assert match_eigs(res.lam, orc.lam) < 1e-10
    assert abs(res.iterations - orc.iters) <= 1
    F.close()


def test_iterate_split_full_size():
    """n = 4096 complex-symmetric generalized pencil (q = 24, m0 = 64): the m eigenvalues inside to
    1e-10 of the golden spectrum, iterations within one of the plain FP32 factors'."""
    g = golden_spectrum("c1")
    P = pencils.c1(radius=g["radius"])
    U0 = upload(pencils.start_block(1, P.n, P.m0))
    A, B = upload(P.A), upload(P.B)
    its = {}
    for split in (True, False):
        F = fm().Feast(A, B, P.center, P.radius, 1.0, P.q, P.m0, precision="fp32", split_update=split)
        res = F.iterate(U0)
        assert res.converged and len(res.lam) == g["m"]
        assert match_eigs(res.lam, g["nearest"][: g["m"]]) < 1e-10
        assert np.all(res.resid <= 1e-10)
        its[split] = res.iterations
        F.close()
    assert abs(its[True] - its[False]) <= 1


def test_batch_split_matches_single():
    """A batch of pencils of different orders with split updates: the same eigenvalues as the single
    contexts with split updates, bit for bit in the factorisation-dependent results."""
    sizes = [130, 257, 300, 520]
    pens = [random_pencil(n, seed=n, with_B=True, m=6) for n in sizes]
    U0s = [pencils.complex_gaussian(np.random.default_rng(n), (n, 10)) for n in sizes]
    mats = [(upload(A), upload(B)) for A, B, _ in pens]
    b = fm().FeastBatch(mats, (0j, 1.0, 1.0), m0=10, q=16, precision="fp32", split_update=True)
    res, rcs = b.iterate([upload(u) for u in U0s])
    b.close()
    for (A, B, lam), (Ad, Bd), U0, r in zip(pens, mats, U0s, res):
        ref = brute.eigenvalues_inside(lam, 0j, 1.0)
        assert r.converged and len(r.lam) == len(ref)
        assert match_eigs(r.lam, ref) < 1e-10
        F = fm().Feast(Ad, Bd, 0j, 1.0, 1.0, 16, 10, precision="fp32", split_update=True)
        s = F.iterate(upload(U0))
        F.close()
        assert np.array_equal(np.sort_complex(s.lam), np.sort_complex(r.lam))
