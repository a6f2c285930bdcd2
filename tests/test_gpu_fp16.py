"""FP16-update mode (FP32 storage and panels, trailing updates on FP16 matrix cores, FP64
refinement) against the oracle: the unrefined solves carry the error level of the oracle's FP16
emulation, the refined solves and the iteration reach FP64 accuracy."""
import numpy as np
import pytest
import scipy.linalg

import pencils
from oracle import brute, feast, lowprec
from oracle import quadrature as Q
from tests.gpu_common import device, match_eigs, random_pencil, rel_err

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53
U16 = 2.0 ** -11


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


def host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("n", [65, 200, 257, 520])
def test_unrefined_solve_matches_fp16_emulation_level(n):
    """ir_max = 0 returns the plain solve with the FP16-update factors: its error against the FP64
    solve is of the size the oracle's emulation of the same factorisation gives (FP16 level, far
    above FP32), node by node."""
    A, B, lam = random_pencil(n, seed=n + 7, with_B=True, cond=3.0)
    q, m0 = 8, 6
    # partial pivoting: the emulation factors with LAPACK's pivots
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, precision="fp16", ir_max=0, pivoting="partial")
    F32 = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, precision="fp32", ir_max=0, pivoting="partial")
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", q)
    rhs = pencils.complex_gaussian(np.random.default_rng(n), (n, m0))
    rd = upload(rhs)
    for k in (0, 3):
        T = feast.node_matrix(A, B, z[k])
        exact = scipy.linalg.lu_solve(scipy.linalg.lu_factor(T), rhs)
        emu = scipy.linalg.lu_solve(lowprec.factor_fp16_scaled(T), rhs.astype(np.complex64))
        e_emu = rel_err(emu, exact)
        e_gpu = rel_err(host(F.node_solve(k, rd)), exact)
        e_32 = rel_err(host(F32.node_solve(k, rd)), exact)
        if n > 64:   # a trailing update exists
            assert 0.1 * e_emu < e_gpu < 10 * e_emu, (k, e_gpu, e_emu)
            assert e_gpu > 20 * e_32, (k, e_gpu, e_32)
        else:
            assert e_gpu < 10 * e_emu + 1e-6
    F.close()
    F32.close()


def structured_node(n, seed):
    """T = L0 U0 with L0 unit lower triangular (strictly lower part complex Gaussian / sqrt(n), so
    |re| + |im| of every multiplier is well below 1/2) and U0 upper triangular with diagonal moduli
    in [1, 2]: partial pivoting keeps every diagonal pivot with a margin above 2 in the |re| + |im|
    metric, which FP16-level changes of the trailing matrix cannot overturn, so the library and the
    emulation factor with the same (identity) pivot sequence."""
    g = np.random.default_rng(seed)
    L = np.tril(pencils.complex_gaussian(g, (n, n)), -1) / np.sqrt(n) + np.eye(n)
    d = (1.0 + g.uniform(0, 1, n)) * np.exp(2j * np.pi * g.uniform(0, 1, n))
    U = np.triu(pencils.complex_gaussian(g, (n, n)), 1) / np.sqrt(n) + np.diag(d)
    return L @ U


@pytest.mark.parametrize("n", [65, 257, 520, 1100])
def test_fp16_factor_solves_match_emulation_elementwise(n):
    """Partial pivoting, ir_max = 0: solves with the library's FP16-update factors against solves
    with the oracle's emulation of the same factorisation (lowprec.factor_fp16_scaled: FP32 panels,
    U12 of each step scaled by a power of two, FP16 operands, FP32 accumulation), entry by entry.

    Why structured node matrices: on general matrices the FP16 roundings change the trailing matrix
    by u16-relative amounts, enough to change later pivot choices, so two correct FP16
    factorisations (or the emulation and the same emulation of T (1 + 1e-9 G)) follow different
    pivot sequences and differ by as much as either differs from the exact solve.  Here node 0 is
    T = L0 U0 (structured_node), whose pivots are unambiguous.

    Bounds.  (1) Every entry of the library's solve is within the FP16 forward-error level
    kappa(T) u16 sqrt(n / 64) (sum of n / 64 update roundings of relative size u16) of the
    emulation's.  (2) Where few updates run, the library rounds the same operands as the emulation:
    their difference is a small fraction of either one's error (measured on the CPU, the emulation
    against itself on T (1 + 1e-7 G): 0.03 at n = 65, 0.2-0.3 at n = 257-520; the fraction grows
    with n because each update's roundings move the next steps' operands by u16-relative amounts).
    A library that scaled L21 instead of U12, dropped the scale-back, accumulated in FP16 or skipped
    the rounding would differ from the emulation as much as from the exact solve or more.  (3) The
    solve error is of FP16 size, far above an FP32 factorisation's."""
    T = structured_node(n, n)
    q, m0 = 8, 6
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", q)
    A = np.asfortranarray(z[0] * np.eye(n) - T)      # node 0: z_0 I - A = T
    rhs = pencils.complex_gaussian(np.random.default_rng(n), (n, m0))
    kappa = np.linalg.cond(T)
    exact = np.linalg.solve(T, rhs)
    emu = scipy.linalg.lu_solve(lowprec.factor_fp16_scaled(T), rhs.astype(np.complex64)).astype(np.complex128)
    F = fm().Feast(upload(A), None, 0j, 1.0, 1.0, q, m0, precision="fp16", ir_max=0, pivoting="partial")
    F32 = fm().Feast(upload(A), None, 0j, 1.0, 1.0, q, m0, precision="fp32", ir_max=0, pivoting="partial")
    rd = upload(rhs)
    gpu = host(F.node_solve(0, rd))
    g32 = host(F32.node_solve(0, rd))
    F.close()
    F32.close()
    scale = np.abs(exact).max()
    d_emu = np.abs(emu - exact).max() / scale
    d_pair = np.abs(gpu - emu).max() / scale
    d_32 = np.abs(g32 - exact).max() / scale
    print(f"n={n} kappa={kappa:.1f} emu-exact {d_emu:.2e} gpu-emu {d_pair:.2e} ratio {d_pair / d_emu:.3f} "
          f"fp32-exact {d_32:.2e}")
    assert np.all(np.abs(gpu - emu) <= kappa * U16 * np.sqrt(n / 64.0) * scale), d_pair
    if n <= 64 + 1:
        assert d_pair <= 0.15 * d_emu, (d_pair, d_emu)
    elif n <= 520:
        assert d_pair <= 0.6 * d_emu, (d_pair, d_emu)
    assert d_pair <= 1.5 * d_emu, (d_pair, d_emu)
    assert d_emu > 20 * d_32 and np.abs(gpu - exact).max() / scale > 20 * d_32


@pytest.mark.parametrize("n", [200, 520])
@pytest.mark.parametrize("side", [0, 1])
def test_refined_solve_reaches_fp64(n, side):
    A, B, lam = random_pencil(n, seed=3 * n, with_B=True, cond=3.0)
    q, m0 = 8, 5
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, q, m0, precision="fp16", ir_max=30)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", q)
    rhs = pencils.complex_gaussian(np.random.default_rng(n + 1), (n, m0))
    for k in (1, 5):
        T = feast.node_matrix(A, B, z[k])
        ref = scipy.linalg.lu_solve(scipy.linalg.lu_factor(T), rhs, trans=2 if side else 0)
        tol = 200 * np.linalg.cond(T) * U64 * max(1, np.sqrt(n) / 4)
        got = host(F.node_solve(k, upload(rhs), side))
        assert rel_err(got, ref) < tol, (k, rel_err(got, ref), tol)
    F.close()


def test_ill_conditioned_nodes_escalate_and_stay_accurate():
    """Node systems with kappa u16 > 1 stall the FP16 refinement: the filter is repeated with FP32
    factorisations and still matches the oracle's FP64 filter."""
    A, B, lam = random_pencil(300, seed=11, with_B=True, cond=1e3)
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, 16, 12, precision="fp16")
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", 16)
    U = pencils.complex_gaussian(np.random.default_rng(2), (300, 12))
    ref = feast.filter_right(feast.factor_nodes(A, B, z), s, B, U)
    kappa = max(np.linalg.cond(feast.node_matrix(A, B, zk)) for zk in z)
    assert kappa * 2.0 ** -11 > 1
    got = host(F.filter(upload(U)))
    assert rel_err(got, ref) < 200 * kappa * U64 * 5
    F.close()


@pytest.mark.parametrize("variant", ["R", "Bi"])
def test_iterate_fp16(variant):
    """The iteration in FP16 mode reaches the prescribed in-contour spectrum to 1e-10 (with FP32
    factorisations substituted if the FP16 ones stall it)."""
    P = pencils.c0()
    U0 = pencils.start_block(0, P.n, P.m0)
    F = fm().Feast(upload(P.A), None, P.center, P.radius, 1.0, P.q, P.m0, precision="fp16", variant=variant)
    res = F.iterate(upload(U0))
    ref = brute.eigenvalues_inside(P.lam, P.center, P.radius)
    assert res.converged, res.history
    assert len(res.lam) == len(ref)
    assert match_eigs(res.lam, ref) < 1e-10
    assert np.all(res.resid <= 1e-10)
    F.close()


def test_iterate_fp16_well_conditioned_without_escalation():
    """A pencil whose node systems suit FP16 factors converges without the FP32 fallback."""
    A, B, lam = random_pencil(400, seed=21, with_B=True, m=8, cond=2.0)
    U0 = pencils.complex_gaussian(np.random.default_rng(3), (400, 16))
    F = fm().Feast(upload(A), upload(B), 0j, 1.0, 1.0, 16, 16, precision="fp16")
    res = F.iterate(upload(U0))
    assert res.converged, res.history
    assert not res.escalated
    assert match_eigs(res.lam, brute.eigenvalues_inside(lam, 0j, 1.0)) < 1e-10
    F.close()


def test_batch_fp16_matches_single():
    import torch
    P = [pencils.c2_pencil(j, n, m) for j, (n, m) in enumerate([(300, 9), (129, 5), (520, 20)])]
    dev = [(upload(p.A), upload(p.B)) for p in P]
    batch = fm().FeastBatch(dev, (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16, precision="fp16", ir_max=0)
    for j, p in enumerate(P):
        U = upload(pencils.start_block(2, p.n, p.m0, salt=7 + j))
        single = fm().Feast(dev[j][0], dev[j][1], 0j, 1.0, 1.0, 16, p.m0, precision="fp16", ir_max=0)
        a = batch.member_filter(j, U)
        b = single.filter(U)
        torch.cuda.synchronize()
        assert torch.equal(a, b), j
        single.close()
    batch.close()
