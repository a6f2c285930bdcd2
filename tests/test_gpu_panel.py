"""Panel kernels.  With partial pivoting the three kernels (register, sweeping, multi-workgroup)
perform the same operations in the same order, so the factorisations and every solve agree bit for
bit whichever variant the tuning selects; the autotuner measures and records their crossover.
Tournament pivoting (an option) chooses other pivot rows, so its solves are
checked against the oracle's partial-pivoting solves to the conditioning bound, at sizes whose
reduction tree has one to six levels."""
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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [300, 700])
def test_panel_variants_agree_bitwise(prec, n):
    import torch
    A, B, lam = random_pencil(n, seed=n, with_B=True)
    Ad, Bd = fm().to_device(A, device()), fm().to_device(B, device())
    U = fm().to_device(pencils.complex_gaussian(np.random.default_rng(1), (n, 12)), device())
    outs = []
    try:
        for rows in (0, 1 << 20):   # multi-workgroup above the register panel / sweeping everywhere
            fm().set_panel_rows(prec, 8, rows)
            F = fm().Feast(Ad, Bd, 0j, 1.0, 1.0, 8, 12, precision=prec, pivoting="partial")
            outs.append(F.filter(U).clone())
            F.close()
    finally:
        fm().set_panel_rows(prec, 8, 0)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", 8)
    ref = feast.filter_right(feast.factor_nodes(A, B, z), s, B, pencils.complex_gaussian(np.random.default_rng(1), (n, 12)))
    assert rel_err(outs[0].cpu().numpy(), ref) < 1e-9


def test_autotune_records_crossover(tmp_path):
    path = tmp_path / "tune.txt"
    rows, table = fm().autotune("fp32", 16, cache_path=path, device=device())
    assert rows in [64, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096, 6144]
    assert np.all(table[:, 1] > 0) and np.all(table[:, 2] > 0)
    line = [l.split() for l in path.read_text().splitlines()]
    assert ["1", "16", str(rows)] in line
    fm().set_panel_rows("fp32", 16, 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [300, 700, 1100, 2500])
def test_tournament_pivoting_solves_match_oracle(prec, n):
    import scipy.linalg
    A, B, lam = random_pencil(n, seed=2 * n + 1, with_B=True, m=max(1, n // 50))
    q, m0 = 8, 6
    F = fm().Feast(fm().to_device(A, device()), fm().to_device(B, device()), 0j, 1.0, 1.0, q, m0, precision=prec,
                   pivoting="tournament")
    Fp = fm().Feast(fm().to_device(A, device()), fm().to_device(B, device()), 0j, 1.0, 1.0, q, m0, precision=prec,
                    pivoting="partial")
    z, s = Q.nodes_and_weights(0j, 1.0, 1.0, "trapezoid", q)
    rhs = pencils.complex_gaussian(np.random.default_rng(n), (n, m0))
    rd = fm().to_device(rhs, device())
    for k in (0, 5):
        T = feast.node_matrix(A, B, z[k])
        kappa = np.linalg.cond(T) if n <= 1100 else 1e4
        for side in (0, 1):
            ref = scipy.linalg.lu_solve(scipy.linalg.lu_factor(T), rhs, trans=2 if side else 0)
            tol = (50 if prec == "fp64" else 200) * kappa * 2.0 ** -53 * max(1, np.sqrt(n) / 4)
            for G in (F, Fp):
                got = G.node_solve(k, rd, side).cpu().numpy()
                assert rel_err(got, ref) < tol, (k, side, rel_err(got, ref), tol)
    F.close()
    Fp.close()


def test_tournament_pivoting_reports_zero_pivot():
    """A tall panel with an exactly zero column (an eigenvalue on node 0): FEAST_ESINGULAR + 0."""
    n = 600
    d = np.linspace(1.5, 3.0, n).astype(np.complex128)
    d[7] = 1.0
    with pytest.raises(fm().FeastError) as e:
        fm().Feast(fm().to_device(np.asfortranarray(np.diag(d)), device()), None, 0j, 1.0, 1.0, 16, 4,
                   pivoting="tournament")
    assert e.value.code == fm().binding.FEAST_ESINGULAR + 0


@pytest.mark.parametrize("variant", ["R", "Bi"])
def test_tournament_pivoting_iteration(variant):
    """The whole iteration with tournament-pivoted factorisations reaches the prescribed spectrum."""
    from oracle import brute
    from tests.gpu_common import match_eigs
    A, B, lam = random_pencil(900, seed=5, with_B=True, m=12)
    U0 = pencils.complex_gaussian(np.random.default_rng(4), (900, 20))
    F = fm().Feast(fm().to_device(A, device()), fm().to_device(B, device()), 0j, 1.0, 1.0, 16, 20, variant=variant,
                   precision="fp32", pivoting="tournament")
    r = F.iterate(fm().to_device(U0, device()))
    assert r.converged and match_eigs(r.lam, brute.eigenvalues_inside(lam, 0j, 1.0)) < 1e-10
    F.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16", "fp64"])
def test_update_tile_shapes_agree_and_the_tuner_sets_the_table(prec):
    """Every compiled tile shape of a trailing-update kernel sums each output in the same order (the
    same operand slices, the same matrix-core steps), so factorisations made with any of them give
    bit-identical filters; the tuner then picks a shape per row bucket, sets the table and reports a
    throughput for every shape it timed.  The tables: "fp32" the split FP16 kernel of the FP32 mode,
    "fp16" the FP32 matrix-core kernel (FP32 contexts with split_update off), "fp64" the FP64 kernel."""
    import torch
    from tests.gpu_common import random_pencil
    fmod = fm()
    A, B, lam = random_pencil(700, 31, True)
    dA, dB = fmod.to_device(A, device()), fmod.to_device(B, device())
    U = fmod.to_device(pencils.start_block(2, 700, 12, salt=5), device())
    shapes = fmod.binding.TILE_SHAPES[prec]
    ctx = {"fp32": dict(precision="fp32"), "fp16": dict(precision="fp32", split_update=False),
           "fp64": dict(precision="fp64")}[prec]
    outs = []
    for t in range(len(shapes)):
        for b in range(6):
            fmod.binding.set_update_tile(prec, b, t)
        with fmod.Feast(dA, dB, 0j, 1.0, 1.0, 16, 12, **ctx) as F:
            outs.append(F.filter(U).clone())
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    table = fmod.binding.autotune_tiles(prec, 16, device=device())
    assert len(table) == 6
    for rows, shape, tf in table:
        assert shape in shapes and set(tf) == set(shapes) and all(v > 0 for v in tf.values())
    for b in range(6):
        fmod.binding.set_update_tile(prec, b, 0)
