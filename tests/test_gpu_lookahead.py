"""Lookahead of the factorisation: the next panel is factored on a second stream while the rest of
the trailing update runs.  The two parts of the update and the panel touch disjoint entries, and every
kernel performs the same arithmetic in the same order, so the factors (and every solve) equal those
of the one-stream sequence bit for bit, for single pencils, captured batches and every precision."""
import numpy as np
import pytest

import pencils
from oracle import feast
from oracle import quadrature as Q
from tests.gpu_common import device, random_pencil, rel_err

pytestmark = pytest.mark.gpu


def fm():
    import paper_1404_2891_amd as m
    return m


def upload(a):
    return None if a is None else fm().to_device(a, device())


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("n", [65, 130, 700, 1500])
def test_lookahead_factors_bitwise_equal(prec, n):
    import torch
    A, B, lam = random_pencil(n, seed=n + 3, with_B=True, cond=3.0)
    Ad, Bd = upload(A), upload(B)
    U0 = pencils.complex_gaussian(np.random.default_rng(n), (n, 10))
    U = upload(U0)
    outs = []
    for la in (True, False):
        F = fm().Feast(Ad, Bd, 0j, 1.0, 1.0, 8, 10, precision=prec, ir_max=0, lookahead=la)
        outs.append([F.filter(U, side).clone() for side in (0, 1)])
        F.close()
    torch.cuda.synchronize()
    for side in (0, 1):
        assert torch.equal(outs[0][side], outs[1][side]), (prec, n, side)
    if prec == "fp64":
        z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", 8)
        ref = feast.filter_right(feast.factor_nodes(A, B, z), s, B, U0)
        assert rel_err(outs[0][0].cpu().numpy(), ref) < 1e-9


def test_lookahead_tournament_bitwise_equal():
    import torch
    n = 1100
    A, B, lam = random_pencil(n, seed=17, with_B=True)
    Ad, Bd = upload(A), upload(B)
    U = upload(pencils.complex_gaussian(np.random.default_rng(4), (n, 8)))
    outs = []
    for la in (True, False):
        F = fm().Feast(Ad, Bd, 0j, 1.0, 1.0, 8, 8, precision="fp32", ir_max=0, pivoting="tournament", lookahead=la)
        outs.append(F.filter(U).clone())
        F.close()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lookahead_batch_graph_bitwise_equal(prec):
    """The batch graph captures the fork and join; its members equal the one-stream graph's."""
    import torch
    sizes = [(300, 9), (64, 3), (1100, 20), (129, 5), (700, 12)]
    P = [pencils.c2_pencil(j, n, m) for j, (n, m) in enumerate(sizes)]
    dev = [(upload(p.A), upload(p.B)) for p in P]
    outs = []
    for la in (True, False):
        batch = fm().FeastBatch(dev, (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16, precision=prec, ir_max=0,
                                lookahead=la)
        res = []
        for j, p in enumerate(P):
            U = upload(pencils.start_block(2, p.n, p.m0, salt=11 + j))
            res.append(batch.member_filter(j, U).clone())
        outs.append(res)
        batch.close()
    torch.cuda.synchronize()
    for j in range(len(P)):
        assert torch.equal(outs[0][j], outs[1][j]), j
