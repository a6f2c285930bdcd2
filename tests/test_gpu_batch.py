"""Batches of pencils (one graph launch for every factorisation, iteration in lockstep) against the
same pencils run one at a time and against the prescribed spectra.

The batch runs the same kernels on every (pencil, node) pair as a pencil set up alone, so the
factorisations, the filters and the converged eigenvalues are compared bit for bit; the spectra
are checked to 1e-10 relative (the FP64-path bound) against the eigenvalues each pencil was built
with (B^-1 A = V diag(lam) V^-1).
"""
import numpy as np
import pytest

import pencils
from oracle import brute, feast
from oracle import quadrature as Q
from tests.gpu_common import device, match_eigs, rel_err

pytestmark = pytest.mark.gpu


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


# orders spanning several factorisation blocks, a ragged tail, a single block and a multi-panel case
SIZES = [300, 64, 129, 520, 257, 70, 1000, 256]
MS = [9, 3, 12, 20, 16, 5, 24, 8]


def batch_pencils(count=len(SIZES)):
    return [pencils.c2_pencil(j, SIZES[j], MS[j]) for j in range(count)]


@pytest.fixture(scope="module")
def small_batch():
    return batch_pencils()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_single_pencils(small_batch, prec):
    import torch
    P = small_batch
    dev = [(upload(p.A), upload(p.B)) for p in P]
    batch = fm().FeastBatch(dev, (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16, precision=prec)
    assert batch.factor_ms() > 0
    U0s = [upload(pencils.start_block(2, p.n, p.m0, salt=10**6 + j)) for j, p in enumerate(P)]
    # filters of the batch members equal those of each pencil set up alone, bit for bit
    for j, p in enumerate(P):
        single = fm().Feast(dev[j][0], dev[j][1], 0j, 1.0, 1.0, 16, p.m0, precision=prec)
        for side in (0, 1):
            a = batch.member_filter(j, U0s[j], side)
            b = single.filter(U0s[j], side)
            torch.cuda.synchronize()
            assert torch.equal(a, b), (j, p.n, side)
        single.close()
    # the lockstep iteration reaches every pencil's prescribed in-contour spectrum
    results, rcs = batch.iterate(U0s)
    assert list(rcs) == [0] * len(P)
    for j, (p, r) in enumerate(zip(P, results)):
        ref = brute.eigenvalues_inside(p.lam, 0j, 1.0)
        assert r.converged, (j, r.history)
        assert len(r.lam) == p.m == len(ref)
        assert match_eigs(r.lam, ref) < 1e-10, (j, match_eigs(r.lam, ref))
        assert np.all(r.resid <= 1e-10)
    # and equals the single-pencil iteration exactly
    for j in (0, 3, 6):
        p = P[j]
        single = fm().Feast(dev[j][0], dev[j][1], 0j, 1.0, 1.0, 16, p.m0, precision=prec)
        s = single.iterate(U0s[j])
        assert s.iterations == results[j].iterations
        assert np.array_equal(s.lam, results[j].lam), (j, s.lam - results[j].lam)
        single.close()
    batch.close()


def test_batch_bi_feast_and_identity_B(small_batch):
    """Bi-FEAST over a batch that mixes pencils with B and with B = I."""
    P = small_batch[:5]
    dev = [(upload(p.A), upload(p.B) if j % 2 else None) for j, p in enumerate(P)]
    # B = I members use B^-1 A as their A, so that the spectrum stays the prescribed one
    for j, p in enumerate(P):
        if j % 2 == 0:
            dev[j] = (upload(np.linalg.solve(p.B, p.A)), None)
    batch = fm().FeastBatch(dev, (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16, variant="Bi")
    U0s = [upload(pencils.start_block(2, p.n, p.m0, salt=10**6 + j)) for j, p in enumerate(P)]
    results, rcs = batch.iterate(U0s)
    for j, (p, r) in enumerate(zip(P, results)):
        ref = brute.eigenvalues_inside(p.lam, 0j, 1.0)
        assert r.converged and len(r.lam) == len(ref), (j, r.history)
        assert match_eigs(r.lam, ref) < 1e-9, (j, match_eigs(r.lam, ref))
        assert r.Y is not None
    batch.close()


def test_batch_contours_differ_per_pencil(small_batch):
    """Each pencil has its own circle (shifted centre, own radius, hence own nodes and weights) that
    holds the same prescribed eigenvalues: |lam| < 0.8 lies inside every circle |z - c| < R with
    |c| = 0.1, R >= 1, and |lam| > 1.5 outside it."""
    P = small_batch[:4]
    dev = [(upload(p.A), upload(p.B)) for p in P]
    contours = [(0.1 * np.exp(2j * np.pi * j / 4), 1.0 + 0.05 * j, 1.0) for j in range(4)]
    refs = [brute.eigenvalues_inside(p.lam, c, R) for p, (c, R, a) in zip(P, contours)]
    assert [len(r) for r in refs] == [p.m for p in P]
    batch = fm().FeastBatch(dev, contours, m0=[p.m0 for p in P], q=16)
    U0s = [upload(pencils.start_block(2, p.n, p.m0, salt=10**6 + j)) for j, p in enumerate(P)]
    results, rcs = batch.iterate(U0s)
    for j, r in enumerate(results):
        assert r.converged and len(r.lam) == len(refs[j]), (j, len(r.lam), len(refs[j]), r.history)
        assert match_eigs(r.lam, refs[j]) < 1e-10
    batch.close()


def test_batch_reports_singular_member():
    """A member with an eigenvalue exactly on node 0 (z_0 = 1) fails setup with FEAST_ESINGULAR + 0 in
    its info slot; the other members report 0."""
    n = 96
    d = np.linspace(1.5, 3.0, n).astype(np.complex128)
    d[7] = 1.0
    good = pencils.c2_pencil(0, 80, 4)
    dev = [(upload(good.A), upload(good.B)), (upload(np.asfortranarray(np.diag(d))), None)]
    with pytest.raises(fm().FeastError) as e:
        fm().FeastBatch(dev, (0j, 1.0, 1.0), m0=[good.m0, 4], q=16)
    assert e.value.code == fm().binding.FEAST_ESINGULAR + 0
    assert list(e.value.info) == [0, fm().binding.FEAST_ESINGULAR + 0]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_member_calls_are_ordered_on_the_batch_stream(prec):
    """Members run on streams of their own; a member's filter starts after work already on the
    caller's stream and the caller's stream waits for it, so its output can be read (cloned) on that
    stream at once, with no device-wide synchronisation in between."""
    sizes = [(300, 9), (64, 3), (1100, 20), (129, 5), (700, 12)]
    P = [pencils.c2_pencil(j, n, m) for j, (n, m) in enumerate(sizes)]
    dev = [(upload(p.A), upload(p.B)) for p in P]
    batch = fm().FeastBatch(dev, (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16, precision=prec, ir_max=0)
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", 16)
    for j, p in enumerate(P):
        U0 = pencils.start_block(2, p.n, p.m0, salt=11 + j)
        got = batch.member_filter(j, upload(U0)).clone().cpu().numpy()
        ref = feast.filter_right(feast.factor_nodes(p.A, p.B, z), s, p.B, U0)
        kappa = max(np.linalg.cond(feast.node_matrix(p.A, p.B, zk)) for zk in z)
        tol = 200 * kappa * 2.0 ** -53 * max(1, np.sqrt(p.n) / 4) * (1 if prec == "fp64" else 2 ** 29)
        assert rel_err(got, ref) < tol, (j, rel_err(got, ref), tol)
    batch.close()
