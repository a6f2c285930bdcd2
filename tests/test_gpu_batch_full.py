"""Batches: the grouped launches of the lockstep iteration against one stream per pencil (same
kernels on the same operands, so bit-identical results), and the full 64-pencil workload (n ~
U{256..2048}, 8-32 prescribed eigenvalues inside the unit circle, q = 16, m0 in {16, 32}) in FP32
(shifted-residual FP64 correction) and FP64 against the eigenvalues each pencil was built with."""
import numpy as np
import pytest

import pencils
from oracle import brute
from tests.gpu_common import device, match_eigs

pytestmark = pytest.mark.gpu


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


SIZES = [300, 64, 129, 520, 257, 70, 1000, 256, 700]
MS = [9, 3, 12, 20, 16, 5, 24, 8, 14]


@pytest.fixture(scope="module")
def small():
    P = [pencils.c2_pencil(j, SIZES[j], MS[j]) for j in range(len(SIZES))]
    return P, [(upload(p.A), upload(p.B)) for p in P]


def _run(dev, P, mode, **kw):
    batch = fm().FeastBatch(dev, (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16, batch_launch=mode, **kw)
    U0s = [upload(pencils.start_block(2, p.n, p.m0, salt=10**6 + j)) for j, p in enumerate(P)]
    res, rcs = batch.iterate(U0s)
    t = batch.timing() if kw.get("timing") else None
    batch.close()
    return res, rcs, t


@pytest.mark.parametrize("prec,variant", [("fp32", "R"), ("fp64", "R"), ("fp32", "Bi"), ("fp64", "L")])
def test_grouped_launches_equal_one_stream_per_pencil(small, prec, variant):
    P, dev = small
    g, rg, _ = _run(dev, P, "grouped", precision=prec, variant=variant)
    s, rs, _ = _run(dev, P, "streams", precision=prec, variant=variant)
    assert list(rg) == list(rs) == [0] * len(P)
    for j in range(len(P)):
        assert g[j].iterations == s[j].iterations, j
        assert np.array_equal(g[j].lam, s[j].lam), (j, np.abs(g[j].lam - s[j].lam).max())
        assert np.array_equal(g[j].resid, s[j].resid), j
        assert np.array_equal(g[j].X.cpu().numpy(), s[j].X.cpu().numpy()), j
        if variant == "Bi":
            assert np.array_equal(g[j].Y.cpu().numpy(), s[j].Y.cpu().numpy()), j
        ref = brute.eigenvalues_inside(P[j].lam, 0j, 1.0)
        assert len(g[j].lam) == len(ref) and match_eigs(g[j].lam, ref) < 1e-9, j


def test_grouped_timing_reports_the_iteration(small):
    """With timing the grouped launches record the solve and Rayleigh-Ritz phases once for the batch
    (flops summed over the pencils), and the host phases add up to the iteration's wall time."""
    P, dev = small
    res, rcs, t = _run(dev, P, "grouped", precision="fp32", timing=True)
    assert list(rcs) == [0] * len(P)
    iters = max(r.iterations for r in res)
    assert t["solve"]["launches"] >= iters and t["solve"]["ms"] > 0
    want = sum(8.0 * p.n * p.n * p.m0 * 16 * r.iterations for p, r in zip(P, res))
    assert t["solve"]["flops"] == pytest.approx(want, rel=1e-12)
    assert t["rayleigh_ritz"]["ms"] > 0
    for k in ("host_reduced_eig", "host_driver", "host_wait"):
        assert t[k]["ms"] > 0, k
    # the orthonormalisation factors its Gram matrices on the device: no host Cholesky phase
    assert t["host_cholesky"]["ms"] == 0


@pytest.fixture(scope="module")
def full_batch():
    """The 64-pencil workload, built on the GPU from the seeded host draws."""
    ns, ms = pencils.c2_sizes(64)
    P = [pencils.c2_pencil(j, ns[j], ms[j], device=device()) for j in range(64)]
    U0s = [upload(pencils.start_block(2, p.n, p.m0, salt=10**6 + j)) for j, p in enumerate(P)]
    return P, U0s


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_full_64_pencil_batch_finds_the_prescribed_spectra(full_batch, prec):
    P, U0s = full_batch
    assert max(p.n for p in P) > 1900 and min(p.n for p in P) < 400
    batch = fm().FeastBatch([(p.A, p.B) for p in P], (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16, precision=prec)
    res, rcs = batch.iterate(U0s)
    batch.close()
    assert list(rcs) == [0] * len(P)
    worst = 0.0
    for j, (p, r) in enumerate(zip(P, res)):
        ref = brute.eigenvalues_inside(p.lam, 0j, 1.0)
        assert r.converged and len(r.lam) == p.m == len(ref), (j, p.n, len(r.lam), p.m, r.history)
        worst = max(worst, match_eigs(r.lam, ref))
        assert np.all(r.resid <= 1e-10), (j, r.resid.max())
    # relative eigenvalue error against the construction (FP64 path bound 1e-10; the FP32 path is
    # corrected in FP64 by the shifted-residual filter and meets the same bound)
    assert worst < 1e-10, worst
    print(f"{prec}: 64 pencils, max relative eigenvalue error {worst:.2e}")
