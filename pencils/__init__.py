"""Seeded synthetic pencils (A, B) and start blocks for non-Hermitian FEAST.

This module only draws random numbers and assembles input matrices.  It holds
none of the eigensolver's arithmetic (no quadrature, no factorisation, no
filter, no Rayleigh-Ritz), so both the CPU oracle and the GPU path can take
their inputs from here without sharing any of the method.

The problem is the generalized eigenproblem A x = lambda B x with n x n
complex A, B, B invertible and B^-1 A diagonalizable (paper, Section 2,
eqn:eigendecomposition).  The paper's own matrices (QC324/QC2534, the Benzene
FEM pencils, the transport pencil) are not available, so these pencils stand
in for them: dense complex non-Hermitian pencils with a prescribed spectrum,
and complex-symmetric pencils with an absorbing (complex) diagonal term as in
the paper's Section 5.5 applications.

Every array is complex128, column-major (Fortran order), so that a torch
tensor made from it with ``torch.from_numpy(M.T).T`` style transposition is not
needed: callers pass ``np.asfortranarray`` data straight to the C-ABI.

Seeds: configuration i uses base seed 140428910 + i; pencil j of a batch uses
``default_rng([base, j])``; the start block uses ``default_rng([base, 10**6])``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 140428910


def base_seed(cfg: int) -> int:
    return BASE_SEED + cfg


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """i.i.d. complex Gaussian with E|g|^2 = 1 (real and imaginary parts ~ N(0, 1/2))."""
    s = math.sqrt(0.5)
    return (rng.standard_normal(shape) * s + 1j * (rng.standard_normal(shape) * s)).astype(np.complex128)


def start_block(cfg: int, n: int, p: int, salt: int = 10**6) -> np.ndarray:
    """Random start block U0 (n x p), column-major complex128."""
    rng = np.random.default_rng([base_seed(cfg), salt])
    return np.asfortranarray(complex_gaussian(rng, (n, p)))


# ---------------------------------------------------------------------------
# spectra
# ---------------------------------------------------------------------------

def uniform_disk(rng, count, radius):
    """Area-uniform points in |z| < radius."""
    r = radius * np.sqrt(rng.random(count))
    th = 2.0 * np.pi * rng.random(count)
    return r * np.exp(1j * th)


def uniform_annulus(rng, count, r_in, r_out):
    """Area-uniform points in r_in < |z| < r_out."""
    u = rng.random(count)
    r = np.sqrt(r_in * r_in + u * (r_out * r_out - r_in * r_in))
    th = 2.0 * np.pi * rng.random(count)
    return r * np.exp(1j * th)


def prescribed_spectrum(rng, n, m, r_inside=0.8, r_in=1.5, r_out=5.0, min_abs=1e-3):
    """m eigenvalues area-uniform in |z| < r_inside and n - m in the annulus r_in < |z| < r_out.

    Inside draws with |z| < min_abs are redrawn so that relative residuals
    ||Ax - lambda Bx|| / (|lambda| ||Bx||) stay well defined."""
    inside = uniform_disk(rng, m, r_inside)
    while m and np.any(np.abs(inside) < min_abs):
        bad = np.abs(inside) < min_abs
        inside[bad] = uniform_disk(rng, int(bad.sum()), r_inside)
    outside = uniform_annulus(rng, n - m, r_in, r_out)
    return np.concatenate([inside, outside])


def clipped_gaussian_basis(rng, n, cond_max=1e3):
    """Complex Gaussian V whose singular values are clipped to sigma_1 / cond_max (cond(V) <= cond_max)."""
    G = complex_gaussian(rng, (n, n))
    Us, s, Wh = np.linalg.svd(G)
    s2 = np.maximum(s, s[0] / cond_max)
    if np.all(s2 == s):
        return G
    return (Us * s2) @ Wh


def gaussian_singular_values(rng, n):
    """Singular values (descending) of an n x n complex Gaussian matrix (E|g|^2 = 1), drawn without
    forming it: Householder bidiagonalisation shows that such a matrix has the singular values of
    the real bidiagonal matrix with diagonal chi_{2(n-i)}/sqrt(2), i = 0..n-1, and superdiagonal
    chi_{2(n-1-i)}/sqrt(2), i = 0..n-2 (the chi bidiagonal model of Dumitriu and Edelman).  They
    are the square roots of the eigenvalues of the tridiagonal D^T D."""
    import scipy.linalg
    d = np.sqrt(rng.chisquare(2.0 * np.arange(n, 0, -1)) / 2.0)
    e = np.sqrt(rng.chisquare(2.0 * np.arange(n - 1, 0, -1)) / 2.0) if n > 1 else np.zeros(0)
    diag = d * d + np.concatenate([[0.0], e * e])
    w = scipy.linalg.eigvalsh_tridiagonal(diag, d[:-1] * e) if n > 1 else diag
    return np.sqrt(np.maximum(w, 0.0))[::-1]


def haar_unitary(G, xp=np):
    """Haar-distributed unitary from a complex Gaussian G: Q of G = QR with the phases of diag(R)
    moved into Q (Mezzadri's construction).  xp is numpy or torch."""
    Q, R = xp.linalg.qr(G)
    d = xp.diagonal(R) if xp is np else xp.diagonal(R, 0)
    ph = d / xp.abs(d)
    return Q * ph[None, :]


def factored_gaussian_basis(rng, n, cond_max=1e3, device=None):
    """V with the distribution of clipped_gaussian_basis, as factors (U, s, W) with V = U diag(s) W^H
    and V^-1 = W diag(1/s) U^H: a complex Gaussian matrix is bi-unitarily invariant, so its singular
    vectors are Haar unitaries independent of its singular values, which are drawn through the chi
    bidiagonal model.  With device set (a torch device), the QR factorisations run there and U, W are
    torch tensors."""
    G1 = complex_gaussian(rng, (n, n))
    G2 = complex_gaussian(rng, (n, n))
    s = gaussian_singular_values(rng, n)
    s = np.maximum(s, s[0] / cond_max)
    if device is None:
        return haar_unitary(G1), s, haar_unitary(G2)
    import torch
    U = haar_unitary(torch.from_numpy(G1).to(device), torch)
    W = haar_unitary(torch.from_numpy(G2).to(device), torch)
    return U, torch.from_numpy(s).to(device=device, dtype=torch.complex128), W


@dataclasses.dataclass
class Pencil:
    """A synthetic pencil with its contour and subspace size.

    A, B: n x n complex128, column-major.  B is None for B = I.
    lam: prescribed eigenvalues (None when the spectrum is not prescribed).
    center, radius, aspect: the contour (an ellipse; aspect 1 is a circle).
    q: number of contour nodes (= number of node factorisations).
    m0: subspace size p.  m: number of eigenvalues inside (None if unknown)."""
    A: np.ndarray
    B: Optional[np.ndarray]
    lam: Optional[np.ndarray]
    center: complex
    radius: float
    aspect: float
    q: int
    m0: int
    m: Optional[int]
    name: str = ""

    @property
    def n(self) -> int:
        return self.A.shape[0]

    def B_or_identity(self) -> np.ndarray:
        return np.eye(self.n, dtype=np.complex128) if self.B is None else self.B


def prescribed_pencil(rng, n, lam, B=None, cond_max=1e3):
    """A with B^-1 A = V diag(lam) V^-1 (A = B V diag(lam) V^-1, or V diag(lam) V^-1 if B is None)."""
    V = clipped_gaussian_basis(rng, n, cond_max)
    A = (V * lam) @ np.linalg.inv(V)
    if B is not None:
        A = B @ A
    return np.asfortranarray(A), V


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def c0(n: int = 200, m: int = 10, seed_cfg: int = 0, q: int = 16, m0: int = 16) -> Pencil:
    """Plain FP64 workload: B = I, A = V diag(lam) V^-1 with m eigenvalues in |z| < 0.8 and n - m
    in 1.5 < |z| < 5; unit circle at 0, q trapezoid nodes, m0 = 16."""
    rng = np.random.default_rng([base_seed(seed_cfg), 0])
    lam = prescribed_spectrum(rng, n, m)
    A, _ = prescribed_pencil(rng, n, lam)
    return Pencil(A, None, lam, 0j, 1.0, 1.0, q, m0, m, name=f"c0_n{n}")


def real_pencil(rng, n, m_pairs, m_real, r_inside=0.8, r_in=1.5, r_out=5.0):
    """Real A, B (stored as complex128) with B^-1 A = V D V^-1, D real block diagonal: m_pairs
    conjugate pairs (2 x 2 blocks [[a, b], [-b, a]]) and m_real real eigenvalues area-uniform in
    |z| < r_inside, the rest (pairs, and one real when the count is odd) in r_in < |z| < r_out;
    V = 2 I + G / sqrt(n) and B = I + 0.1 H / sqrt(n) with real Gaussian G, H.  Returns A, B and the
    eigenvalues (block order)."""
    def ring(lo, hi, count, real):
        r = np.sqrt(rng.uniform(lo ** 2, hi ** 2, count))
        if real:
            return r * np.sign(rng.uniform(-1, 1, count))
        return r * np.exp(1j * rng.uniform(0.1, np.pi - 0.1, count))
    inner_pairs, inner_real = ring(0, r_inside, m_pairs, False), ring(0.05, r_inside, m_real, True)
    n_out_pairs = (n - 2 * m_pairs - m_real) // 2
    n_out_real = n - 2 * m_pairs - m_real - 2 * n_out_pairs
    outer_pairs, outer_real = ring(r_in, r_out, n_out_pairs, False), ring(r_in, r_out, n_out_real, True)
    D = np.zeros((n, n))
    lam = []
    i = 0
    for z in np.concatenate([inner_pairs, outer_pairs]):
        D[i:i + 2, i:i + 2] = [[z.real, z.imag], [-z.imag, z.real]]
        lam += [z, np.conj(z)]
        i += 2
    for x in np.concatenate([inner_real, outer_real]):
        D[i, i] = x.real
        lam.append(complex(x.real))
        i += 1
    V = rng.standard_normal((n, n)) / np.sqrt(n) + 2.0 * np.eye(n)
    B = np.eye(n) + 0.1 * rng.standard_normal((n, n)) / np.sqrt(n)
    A = B @ V @ D @ np.linalg.inv(V)
    return np.asfortranarray(A.astype(np.complex128)), np.asfortranarray(B.astype(np.complex128)), np.array(lam)


def complex_symmetric_pencil(rng, n, absorb=0.05, bscale=0.05):
    """A = (G + G^T)/(2 sqrt n) + i diag(absorb (j/n)^2), B = I + bscale (H + H^H)/sqrt n (HPD)."""
    G = complex_gaussian(rng, (n, n))
    A = (G + G.T) / (2.0 * math.sqrt(n))
    del G
    j = np.arange(1, n + 1, dtype=np.float64)
    A[np.diag_indices(n)] += 1j * absorb * (j / n) ** 2
    H = complex_gaussian(rng, (n, n))
    B = bscale * (H + H.conj().T) / math.sqrt(n)
    del H
    B[np.diag_indices(n)] += 1.0
    return np.asfortranarray(A), np.asfortranarray(B)


def c1(n: int = 4096, radius: Optional[float] = None, seed_cfg: int = 1, q: int = 24, m0: int = 64,
       m: Optional[int] = None) -> Pencil:
    """Single complex-symmetric generalized pencil, circle at 0.5+0.2i.

    The radius is an input: the stated radius (0.3) encloses far more
    eigenvalues than m0 = 64 can hold, so the workload uses the radius R*
    placed in the middle of the gap after the 48th eigenvalue nearest to the
    center (computed once from the brute-force spectrum and stored with the
    golden data)."""
    rng = np.random.default_rng([base_seed(seed_cfg), 0])
    A, B = complex_symmetric_pencil(rng, n)
    return Pencil(A, B, None, 0.5 + 0.2j, 0.3 if radius is None else radius, 1.0, q, m0, m, name=f"c1_n{n}")


def c3(n: int = 8192, radius: Optional[float] = None, seed_cfg: int = 3, q: int = 32, m0: int = 128,
       m: Optional[int] = None) -> Pencil:
    """The same construction as c1 with its own seed; circle at 0, 32 nodes, m0 = 128."""
    rng = np.random.default_rng([base_seed(seed_cfg), 0])
    A, B = complex_symmetric_pencil(rng, n)
    return Pencil(A, B, None, 0j, 0.5 if radius is None else radius, 1.0, q, m0, m, name=f"c3_n{n}")


def real_workload(n: int = 4096, seed_cfg: int = 5, q: int = 24, m0: int = 64, m_pairs: int = 20,
                  m_real: int = 8) -> Pencil:
    """Real generalized pencil for nodes that share a factorisation with their conjugates: 20 pairs and
    8 real eigenvalues inside the unit circle (m = 48), q trapezoid nodes, m0 = 64."""
    rng = np.random.default_rng([base_seed(seed_cfg), 0])
    A, B, lam = real_pencil(rng, n, m_pairs, m_real)
    return Pencil(A, B, lam, 0j, 1.0, 1.0, q, m0, 2 * m_pairs + m_real, name=f"real_n{n}")


def grid_spectrum(rng, n, m_in, region=(-1.0, 1.0, -1.0, 1.0), grid=(6, 6), margin=0.3, r_out=(2.0, 5.0)):
    """Eigenvalues for multi-domain runs: m_in inside the rectangle region = (x0, x1, y0, y1), each in
    a random cell of the gx x gy grid over it and at least margin (fraction of the cell's width and
    height) from that cell's edges; n - m_in area-uniform in r_out[0] < |z| < r_out[1]."""
    x0, x1, y0, y1 = region
    gx, gy = grid
    w, h = (x1 - x0) / gx, (y1 - y0) / gy
    ix = rng.integers(0, gx, m_in)
    iy = rng.integers(0, gy, m_in)
    fx = rng.uniform(margin, 1 - margin, m_in)
    fy = rng.uniform(margin, 1 - margin, m_in)
    inside = (x0 + (ix + fx) * w) + 1j * (y0 + (iy + fy) * h)
    r = np.sqrt(rng.uniform(r_out[0] ** 2, r_out[1] ** 2, n - m_in))
    outside = r * np.exp(2j * np.pi * rng.random(n - m_in))
    return np.concatenate([inside, outside])


def c2_sizes(count: int = 64, seed_cfg: int = 2, n_lo: int = 256, n_hi: int = 2048):
    """(n_i, m_i) of the batched workload: n_i ~ U{n_lo..n_hi}, m_i ~ U{8..32}."""
    rng = np.random.default_rng([base_seed(seed_cfg), 10**6 + 1])
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ms = rng.integers(8, 33, size=count)
    return [int(x) for x in ns], [int(x) for x in ms]


def c2_pencil(j: int, n: int, m: int, seed_cfg: int = 2, q: int = 16, device=None) -> Pencil:
    """Pencil j of the batched workload: B = I + 0.1 (H + H^H)/(2 sqrt n), A = B V diag(lam) V^-1 with
    V distributed as the clipped complex Gaussian basis (cond <= 1e3), built from its factors so that
    no SVD or inverse is formed.  With device set (a torch device) the products run there and A, B
    are column-major complex128 torch tensors on it (same draws, same pencil up to rounding)."""
    rng = np.random.default_rng([base_seed(seed_cfg), j])
    lam = prescribed_spectrum(rng, n, m)
    H = complex_gaussian(rng, (n, n))
    U, sv, W = factored_gaussian_basis(rng, n, 1e3, device)
    m0 = 16 if m <= 16 else 32
    if device is None:
        B = 0.1 * (H + H.conj().T) / (2.0 * math.sqrt(n))
        B[np.diag_indices(n)] += 1.0
        Vl = (U * sv) @ (W.conj().T * lam)           # V diag(lam), V = U diag(s) W^H
        Vinv = (W / sv) @ U.conj().T
        A = B @ (Vl @ Vinv)
        return Pencil(np.asfortranarray(A), np.asfortranarray(B), lam, 0j, 1.0, 1.0, q, m0, m, name=f"c2_{j}_n{n}")
    import torch
    Ht = torch.from_numpy(H).to(device)
    B = 0.1 * (Ht + Ht.conj().T) / (2.0 * math.sqrt(n))
    B.diagonal().add_(1.0)
    lt = torch.from_numpy(lam).to(device)
    Vl = (U * sv[None, :]) @ (W.conj().T * lt[None, :])
    Vinv = (W / sv[None, :]) @ U.conj().T
    A = B @ (Vl @ Vinv)
    col = lambda X: X.T.contiguous().T                # column-major storage
    return Pencil(col(A), col(B), lam, 0j, 1.0, 1.0, q, m0, m, name=f"c2_{j}_n{n}")


def c2(count: int = 64, seed_cfg: int = 2, n_lo: int = 256, n_hi: int = 2048):
    ns, ms = c2_sizes(count, seed_cfg, n_lo, n_hi)
    return [c2_pencil(j, ns[j], ms[j], seed_cfg) for j in range(count)]


def c4_pencil(j: int, n: int = 512, seed_cfg: int = 4, m: Optional[int] = None, q: int = 16,
              m0: int = 64, basis: Optional[int] = None, device=None) -> Pencil:
    """Pencil j of the learned-m0 workload: lam = c + R mu with mu drawn as in c0 (m inside 0.8,
    the rest in 1.5 < |mu| < 5), c area-uniform in |c| < 2, R ~ U[0.2, 1.5], m ~ U{0..48}, B = I.

    basis=None draws the eigenvector basis for this pencil alone (clipped complex Gaussian);
    basis=b takes basis b of a shared pool (c4_basis, distributed the same way), so that large
    training sets need only their spectra drawn.  With device set (a torch device) A is built there
    and returned as a column-major complex128 tensor."""
    rng = np.random.default_rng([base_seed(seed_cfg), j])
    if m is None:
        m = int(rng.integers(0, 49))
    c = complex(uniform_disk(rng, 1, 2.0)[0])
    R = float(rng.uniform(0.2, 1.5))
    mu = prescribed_spectrum(rng, n, m, min_abs=0.0)
    lam = c + R * mu
    if basis is None and device is None:
        A, _ = prescribed_pencil(rng, n, lam)
        return Pencil(A, None, lam, c, R, 1.0, q, m0, m, name=f"c4_{j}_n{n}")
    if basis is None:
        U, sv, W = factored_gaussian_basis(rng, n, 1e3, device)
    else:
        U, sv, W = c4_basis(basis, n, seed_cfg, device)
    if device is None:
        A = np.asfortranarray(((U * sv) @ (W.conj().T * lam)) @ ((W / sv) @ U.conj().T))
    else:
        import torch
        lt = torch.from_numpy(lam).to(device)
        A = ((U * sv[None, :]) @ (W.conj().T * lt[None, :])) @ ((W / sv[None, :]) @ U.conj().T)
        A = A.T.contiguous().T
    return Pencil(A, None, lam, c, R, 1.0, q, m0, m, name=f"c4_{j}_n{n}")


_C4_BASES = {}


def c4_basis(b: int, n: int = 512, seed_cfg: int = 4, device=None):
    """Basis b of the learned-m0 pool as factors (U, s, W), V = U diag(s) W^H (cached per device)."""
    key = (b, n, seed_cfg, str(device))
    if key not in _C4_BASES:
        rng = np.random.default_rng([base_seed(seed_cfg), 3 * 10**6 + b])
        _C4_BASES[key] = factored_gaussian_basis(rng, n, 1e3, device)
    return _C4_BASES[key]


def c4_split(kind: str, count: int):
    """Pencil ids and basis ids of the training ("train") or held-out ("eval") pencils: the two
    sets use disjoint pencil seeds and disjoint basis pools (16 training bases, 4 held-out)."""
    if kind == "train":
        return [(j, j % 16) for j in range(count)]
    return [(10**6 + j, 16 + j % 4) for j in range(count)]


def rademacher_complex(rng, shape) -> np.ndarray:
    """Probe vectors with entries (+-1 +- i)/sqrt 2, E[v v^H] = I."""
    re = rng.integers(0, 2, size=shape) * 2 - 1
    im = rng.integers(0, 2, size=shape) * 2 - 1
    return np.asfortranarray((re + 1j * im) / math.sqrt(2.0))


def probe_block(cfg: int, j: int, n: int, count: int = 8) -> np.ndarray:
    rng = np.random.default_rng([base_seed(cfg), 2 * 10**6 + j])
    return rademacher_complex(rng, (n, count))
