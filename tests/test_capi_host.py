"""CPU tests of the C-ABI library: it loads, exports every declared entry point, and its
host-only logic (quadrature nodes, reduced eigensolver, workspace sizing) matches the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg

import paper_1404_2891_amd as fm
from paper_1404_2891_amd import binding
from oracle import quadrature as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(feast_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = fm.lib()
    decl = declared_functions()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(L, name), name
    assert set(binding.EXPORTED) <= set(decl)


def test_library_is_built_for_gfx950_only():
    out = os.popen(f"/opt/rocm/llvm/bin/clang-offload-bundler --list --type=o "
                   f"--input={fm.library_path()} 2>/dev/null").read()
    if out:
        assert "gfx950" in out and "gfx942" not in out


@pytest.mark.parametrize("rule", ["trapezoid", "gauss-legendre"])
@pytest.mark.parametrize("q", [2, 4, 8, 16, 24, 32, 64])
@pytest.mark.parametrize("c,R,a", [(0j, 1.0, 1.0), (0.5 + 0.2j, 0.3, 1.0), (-1 + 2j, 2.5, 0.4)])
def test_contour_nodes_match_oracle(rule, q, c, R, a):
    z, s = fm.contour_nodes(c, R, a, q, rule)
    zo, so = Q.nodes_and_weights(c, R, a, rule, q)
    # same multiset of nodes, same weight at each node
    for zk, sk in zip(zo, so):
        j = np.argmin(np.abs(z - zk))
        assert abs(z[j] - zk) < 1e-13 * (1 + abs(c) + R)
        assert abs(s[j] - sk) < 1e-14 * (1 + abs(sk)) + 1e-15
    if rule == "trapezoid" and a == 1.0:
        mu = c + R * np.array([0.3, 0.9j, -1.3, 0.5 + 0.5j])
        rho = np.sum(s[None, :] / (z[None, :] - mu[:, None]), axis=1)
        assert np.allclose(rho, 1 / (1 - ((mu - c) / R) ** q), rtol=1e-12)


def test_contour_nodes_reject_bad_input():
    C = binding.make_contour(0j, -1.0, 1.0, 16)
    z = np.zeros(16, dtype=np.complex128)
    assert fm.lib().feast_contour_nodes(ctypes.byref(C), z.ctypes.data, z.ctypes.data) != 0
    C = binding.make_contour(0j, 1.0, 1.0, 7)
    assert fm.lib().feast_contour_nodes(ctypes.byref(C), z.ctypes.data, z.ctypes.data) != 0


def _rand(p, seed):
    g = np.random.default_rng(seed)
    return (g.standard_normal((p, p)) + 1j * g.standard_normal((p, p))) / np.sqrt(2 * p)


@pytest.mark.parametrize("p", [1, 2, 3, 8, 17, 64, 128])
def test_reduced_eig_matches_qz(p):
    Ah = _rand(p, p)
    Bh = np.eye(p) + 0.3 * _rand(p, p + 1)
    lam, W, Z = fm.reduced_eig(Ah, Bh, left=True)
    ref = scipy.linalg.eigvals(Ah, Bh)
    from scipy.optimize import linear_sum_assignment
    C = np.abs(lam[:, None] - ref[None, :])
    r, c = linear_sum_assignment(C)
    assert C[r, c].max() < 1e-11 * max(1, np.abs(ref).max())
    assert np.allclose(np.linalg.norm(W, axis=0), 1.0)
    assert np.linalg.norm(Ah @ W - Bh @ W * lam[None, :]) < 1e-11 * np.sqrt(p)
    assert np.allclose(Z.conj().T @ Bh @ W, np.eye(p), atol=1e-9)
    assert np.linalg.norm(Z.conj().T @ Ah - lam[:, None] * (Z.conj().T @ Bh)) < 1e-8 * np.sqrt(p)


@pytest.mark.parametrize("p,split", [(96, 40), (128, 64), (130, 3)])
def test_reduced_eig_block_triangular(p, split):
    # block upper triangular Ah: the Hessenberg form keeps the zero block, so the QR iteration works on
    # the lower block first with the rows above it updated afterwards, then on the upper block with
    # the columns beyond it updated afterwards; orders >= 64 share these updates over threads
    Ah = _rand(p, p + 7)
    Ah[split:, :split] = 0.0
    Bh = np.eye(p) + 0.2 * _rand(p, p + 8)
    lam, W, Z = fm.reduced_eig(Ah, Bh, left=True)
    for _ in range(4):   # the threaded updates give the same result every time
        lam2, W2, Z2 = fm.reduced_eig(Ah, Bh, left=True)
        assert np.array_equal(lam2, lam) and np.array_equal(W2, W) and np.array_equal(Z2, Z)
    ref = scipy.linalg.eigvals(Ah, Bh)
    from scipy.optimize import linear_sum_assignment
    C = np.abs(lam[:, None] - ref[None, :])
    r, c = linear_sum_assignment(C)
    assert C[r, c].max() < 1e-11 * max(1, np.abs(ref).max())
    assert np.allclose(np.linalg.norm(W, axis=0), 1.0)
    assert np.linalg.norm(Ah @ W - Bh @ W * lam[None, :]) < 1e-11 * np.sqrt(p)
    assert np.allclose(Z.conj().T @ Bh @ W, np.eye(p), atol=1e-9)
    assert np.linalg.norm(Z.conj().T @ Ah - lam[:, None] * (Z.conj().T @ Bh)) < 1e-8 * np.sqrt(p)


def test_reduced_eig_concurrent_callers():
    # calls from several host threads at once (the library's worker threads serve one call at a time;
    # the others run alone) give the results of calls made one after another
    from concurrent.futures import ThreadPoolExecutor
    cases = [(_rand(96 + 8 * k, 50 + k), np.eye(96 + 8 * k) + 0.2 * _rand(96 + 8 * k, 60 + k)) for k in range(6)]
    serial = [fm.reduced_eig(A, B, left=True) for A, B in cases]
    with ThreadPoolExecutor(max_workers=6) as ex:
        for _ in range(3):
            par = list(ex.map(lambda c: fm.reduced_eig(c[0], c[1], left=True), cases))
            for (l0, W0, Z0), (l1, W1, Z1) in zip(serial, par):
                assert np.array_equal(l0, l1) and np.array_equal(W0, W1) and np.array_equal(Z0, Z1)


def test_reduced_eig_triangular_and_repeated():
    # already triangular, with a repeated eigenvalue (diagonalizable: identity block)
    Ah = np.diag([1.0, 1.0, 2.0 + 1j, -3.0]).astype(complex)
    Ah[0, 2] = 0.5
    lam, W = fm.reduced_eig(Ah, np.eye(4))
    assert np.allclose(np.sort_complex(lam), np.sort_complex(np.diag(Ah)), atol=1e-13)
    assert np.linalg.norm(Ah @ W - W * lam[None, :]) < 1e-12


def test_workspace_size_scales():
    C = binding.make_contour(0j, 1.0, 1.0, 16)
    o64 = binding.make_options("fp64")
    o32 = binding.make_options("fp32")
    s64 = fm.workspace_size(200, 16, C, o64, False)
    s32 = fm.workspace_size(200, 16, C, o32, False)
    assert s64 > 16 * 200 * 200 * 16
    assert s32 > 16 * 200 * 200 * 8
    big = fm.workspace_size(4096, 64, binding.make_contour(0j, 1.0, 1.0, 24), o64, True)
    assert 24 * 4096 * 4096 * 16 < big < 1.3 * 24 * 4096 * 4096 * 16
    with pytest.raises(binding.FeastError):
        fm.workspace_size(10, 11, C, o64, False)   # m0 > n


def _batch_size(ns, m0s, qs, opts, has_B):
    count = len(ns)
    C = (binding.Contour * count)(*[binding.make_contour(0j, 1.0, 1.0, q) for q in qs])
    n_arr = (ctypes.c_int * count)(*ns)
    m_arr = (ctypes.c_int * count)(*m0s)
    hb = (ctypes.c_int * count)(*[int(h) for h in has_B])
    out = ctypes.c_size_t(0)
    code = fm.lib().feast_batch_workspace_size(count, ctypes.cast(n_arr, ctypes.c_void_p),
                                               ctypes.cast(m_arr, ctypes.c_void_p), ctypes.cast(C, ctypes.c_void_p),
                                               ctypes.byref(opts), ctypes.cast(hb, ctypes.c_void_p), ctypes.byref(out))
    return code, out.value


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_workspace_is_members_plus_tables(prec):
    """A batch needs every member's own workspace plus the set's descriptor and grouped-product
    tables (a few hundred bytes per factorisation step, a copy per part of the nodes), and with grouped iteration launches (the
    default) the 64 MiB arena of their device tables and staged transfers."""
    ns, m0s = [256, 1000, 65, 2048, 300], [16, 32, 16, 32, 8]
    sizes = {}
    for mode in ("streams", "grouped"):
        o = binding.make_options(prec, batch_launch=mode)
        code, sizes[mode] = _batch_size(ns, m0s, [16] * 5, o, [True] * 5)
        assert code == 0
    o = binding.make_options(prec)
    singles = sum(fm.workspace_size(n, m, binding.make_contour(0j, 1.0, 1.0, 16), o, True) for n, m in zip(ns, m0s))
    total = sizes["streams"]
    # the set's descriptors and grouped-product tables: one copy for the whole nodes and one for each
    # of the parts of them that the factorisation graph runs on branches of their own (up to four)
    assert singles <= total <= singles + 5 * (5 * 256 + 256 * (2 * sum(-(-n // 64) for n in ns) + 5 * 24)) + 4096
    assert sizes["grouped"] == total + (64 << 20)
    # classic refinement sweeps keep one stream per pencil (no arena)
    o = binding.make_options(prec, ir_tol=1e-12)
    code, t = _batch_size(ns, m0s, [16] * 5, o, [True] * 5)
    assert code == 0 and t == (total + (64 << 20) if prec == "fp64" else total)


def test_batch_rejects_mixed_node_counts_and_bad_sizes():
    o = binding.make_options("fp64")
    code, _ = _batch_size([100, 200], [8, 8], [16, 24], o, [False, False])
    assert code == binding.FEAST_EUNSUPPORTED
    code, _ = _batch_size([100, 20], [8, 21], [16, 16], o, [False, False])
    assert code < 0
    out = ctypes.c_size_t(0)
    assert fm.lib().feast_batch_workspace_size(0, None, None, None, ctypes.byref(o), None, ctypes.byref(out)) < 0


def test_m0_rule_and_mlp_sizes():
    """m0 = max(8, ceil(1.25 m) + 4) rounded up to a multiple of 8; the perceptron 19-256-256-1 has
    71,425 parameters."""
    for m_hat, m0 in [(0.0, 8), (-3.0, 8), (2.9, 8), (3.3, 16), (10.0, 24), (48.0, 64), (float("nan"), 8)]:
        assert fm.m0_from_estimate(m_hat) == m0, (m_hat, m0)
    assert fm.lib().feast_mlp_param_count(19, 256) == 256 * 19 + 256 + 256 * 256 + 256 + 256 + 1
    out = ctypes.c_size_t(0)
    assert fm.lib().feast_mlp_workspace_size(19, 256, 1024, ctypes.byref(out)) == 0
    assert out.value >= 4 * (4 * 71425 + 4 * 1024 * 256)


def test_autotune_workspace_size():
    out = ctypes.c_size_t(0)
    assert fm.lib().feast_autotune_workspace_size(16, 1, ctypes.byref(out)) == 0
    assert out.value >= 16 * 6144 * 64 * 8
    assert fm.lib().feast_autotune_workspace_size(0, 1, ctypes.byref(out)) < 0


def test_conjugate_node_sharing_workspace_and_validation():
    """With conj_nodes a node and its conjugate share one factorisation: a contour symmetric about
    the real axis needs about half the factor storage; an asymmetric one is refused (host-side
    checks, no device work)."""
    o_full = binding.make_options(precision="fp64")
    o_real = binding.make_options(precision="fp64", conj_nodes="real")
    o_herm = binding.make_options(precision="fp64", conj_nodes="hermitian")
    sym = binding.make_contour(0.3 + 0j, 1.0, 0.7, 24)
    full = fm.workspace_size(2048, 32, sym, o_full, True)
    half = fm.workspace_size(2048, 32, sym, o_real, True)
    assert half == fm.workspace_size(2048, 32, sym, o_herm, True)
    # trapezoid on an ellipse centered on the real axis: 13 of 24 nodes factored (two real nodes)
    assert 0.5 < half / full < 0.6, half / full
    gl = binding.make_contour(0.3 + 0j, 1.0, 1.0, 24, "gauss-legendre")
    assert fm.workspace_size(2048, 32, gl, o_real, True) < half
    nbytes = ctypes.c_size_t(0)
    off_axis = binding.make_contour(0.3 + 0.1j, 1.0, 1.0, 24)
    rc = fm.lib().feast_workspace_size(2048, 32, ctypes.byref(off_axis), ctypes.byref(o_real), 1, ctypes.byref(nbytes))
    assert rc == binding.FEAST_EUNSUPPORTED
    # a glued contour symmetric about the real axis is accepted, a triangle above it is not
    square = binding.make_contour(q=32, pieces=fm.polygon([-0.5 - 0.5j, 0.5 - 0.5j, 0.5 + 0.5j, -0.5 + 0.5j]))
    assert fm.workspace_size(2048, 32, square, o_herm, True) < fm.workspace_size(2048, 32, square, o_full, True)
    tri = binding.make_contour(q=24, pieces=fm.polygon([0j, 2 + 0j, 1 + 1.5j]))
    rc = fm.lib().feast_workspace_size(2048, 32, ctypes.byref(tri), ctypes.byref(o_herm), 1, ctypes.byref(nbytes))
    assert rc == binding.FEAST_EUNSUPPORTED
    # batches do not take shared conjugate nodes
    ns = (ctypes.c_int * 2)(256, 300)
    ms = (ctypes.c_int * 2)(8, 8)
    Cs = (binding.Contour * 2)(sym, sym)
    rc = fm.lib().feast_batch_workspace_size(2, ns, ms, Cs, ctypes.byref(o_real), None, ctypes.byref(nbytes))
    assert rc == binding.FEAST_EUNSUPPORTED
    bad = binding.make_options(precision="fp64")
    bad.conj_nodes = 3
    assert fm.lib().feast_workspace_size(2048, 32, ctypes.byref(sym), ctypes.byref(bad), 1, ctypes.byref(nbytes)) < 0
