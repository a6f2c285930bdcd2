"""Multi-domain runs on the device: count estimates for the cells of a grid over a region in one
probe batch, a load-balanced partition into rectangles, and one batch over the rectangles; every
eigenvalue of the region is found by exactly one tile (brute-force spectrum)."""
import numpy as np
import pytest

import pencils
from tests.domain_grid import GRID, REGION, grid_spectrum, in_region
from tests.gpu_common import device, match_eigs, random_pencil

pytestmark = pytest.mark.gpu


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


@pytest.mark.parametrize("variant", ["R", "Bi"])
def test_multi_domain_finds_every_eigenvalue_once(variant):
    n, m_in = 400, 48
    lam0 = grid_spectrum(n, m_in, seed=1)
    A, B, lam = random_pencil(n, seed=2, with_B=True, spectrum=lam0)
    probes = upload(pencils.rademacher_complex(np.random.default_rng(7), (n, 8)))
    rects, est, res, rcs = fm().multi_domain(upload(A), upload(B), REGION, probes, grid=GRID, target=12, q=16,
                                             variant=variant, max_iter=60)
    assert list(rcs) == [0] * len(rects)
    assert len(rects) >= 3
    # the tiles cover the region without overlap
    area = sum((r[1] - r[0]) * (r[3] - r[2]) for r in rects)
    assert abs(area - 4.0) < 1e-12
    found = np.concatenate([r.lam for r in res])
    ref = lam0[in_region(lam0)]
    assert len(found) == len(ref) == m_in
    assert match_eigs(found, ref) < 1e-10
    for r, rect in zip(res, rects):
        assert r.converged
        assert np.all((r.lam.real > rect[0]) & (r.lam.real < rect[1]) & (r.lam.imag > rect[2]) & (r.lam.imag < rect[3]))


def test_trace_estimate_of_one_domain():
    """The stochastic count of the whole region with 64 probes and 8 Gauss-Legendre points per side,
    against the 48 eigenvalues inside (the estimate's spread for this pencil is a few counts)."""
    n, m_in = 400, 48
    lam0 = grid_spectrum(n, m_in, seed=1)
    A, B, lam = random_pencil(n, seed=2, with_B=True, spectrum=lam0)
    V = upload(pencils.rademacher_complex(np.random.default_rng(8), (n, 64)))
    b = fm().FeastBatch([(upload(A), upload(B))], [fm().rectangle(*REGION)], m0=64, q=32, rule="gauss-legendre",
                        precision="fp32", ir_max=0)
    est = b.trace_estimates(V)
    b.close()
    assert abs(est[0] - m_in) < 0.25 * m_in, est
