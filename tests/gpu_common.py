"""Helpers shared by the GPU tests (inputs and comparisons only; no method arithmetic)."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return "cuda:0"


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def match_eigs(got, ref):
    """Optimal assignment of two eigenvalue sets (equal counts); max relative error."""
    from scipy.optimize import linear_sum_assignment
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert len(got) == len(ref), (len(got), len(ref))
    if len(ref) == 0:
        return 0.0
    C = np.abs(got[:, None] - ref[None, :]) / np.abs(ref)[None, :]
    r, c = linear_sum_assignment(C)
    return float(C[r, c].max())


def golden_spectrum(name):
    with open(os.path.join(HERE, "golden", f"spectrum_{name}.json")) as f:
        d = json.load(f)
    d["nearest"] = np.array([complex(a, b) for a, b in d["nearest"]])
    d["center"] = complex(*d["center"])
    return d


def random_pencil(n, seed, with_B, m=None, cond=1e2, spectrum=None):
    """Small dense pencil with a prescribed spectrum (B^-1 A = V diag(lam) V^-1): `spectrum` when
    given, else m eigenvalues inside the unit circle and the rest outside."""
    import pencils
    g = np.random.default_rng(seed)
    m = max(1, n // 10) if m is None else m
    lam = pencils.prescribed_spectrum(g, n, min(m, n)) if spectrum is None else np.asarray(spectrum)
    B = None
    if with_B:
        H = pencils.complex_gaussian(g, (n, n))
        B = np.asfortranarray(np.eye(n) + 0.1 * (H + H.conj().T) / (2 * np.sqrt(n))
                              + 0.05 * pencils.complex_gaussian(g, (n, n)) / np.sqrt(n))
    V = pencils.clipped_gaussian_basis(g, n, cond)
    A = (V * lam) @ np.linalg.inv(V)
    if B is not None:
        A = B @ A
    return np.asfortranarray(A), B, lam
