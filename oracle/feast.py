"""Plain FP64 non-Hermitian FEAST (paper Sections 3-5).  Test infrastructure only.

Steps, in the paper's order and notation:

* node systems phi_k B - A, each factored once (LU with partial pivoting,
  LAPACK zgetrf via SciPy) and kept for the whole run (Section 5.5: each
  system is factored just once for the entire iterative process);
* right filter  rho(M) U = sum_k sigma_k (phi_k B - A)^-1 (B U)        (eqn:Rasp);
* left filter   B^-H rho(M)^H B^H V = sum_k conj(sigma_k) (phi_k B - A)^-H (B^H V)
  (eqn:quadf_surMconj; the displayed eqn:Lasp is typeset with the inverse
  around the whole sum, read here as one conjugate-transposed solve per node);
* Algorithm R-FEAST and Algorithm Bi-FEAST (Section 4), with the basis
  orthonormalised after the filter (the stability remark after the
  convergence properties);
* candidates: Ritz pairs inside the domain whose residual
  ||A u - lambda B u|| / ||u|| is at most 1e-4; Res_(k) = max residual and
  trace_(k) = sum of candidate Ritz values are tracked (Section 5 preamble).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg

from .quadrature import RULE_TRAPEZOID, glued_nodes_and_weights, inside, inside_glued, nodes_and_weights

CANDIDATE_RESIDUAL = 1e-4


# ---------------------------------------------------------------------------
# node systems and the filters
# ---------------------------------------------------------------------------

def _B(B, n):
    return np.eye(n, dtype=np.complex128) if B is None else B


def node_matrix(A, B, zk):
    """phi_k B - A."""
    return zk * _B(B, A.shape[0]) - A


def factor_nodes(A, B, z):
    """One LU with partial pivoting per node (zgetrf)."""
    return [scipy.linalg.lu_factor(node_matrix(A, B, zk)) for zk in z]


def solve_nodes(lus, rhs, conj_trans=False):
    """Y_k = (phi_k B - A)^-1 rhs, or (phi_k B - A)^-H rhs."""
    return [scipy.linalg.lu_solve(lu, rhs, trans=2 if conj_trans else 0) for lu in lus]


def filter_right(lus, sigma, B, U):
    """rho(M) U = sum_k sigma_k (phi_k B - A)^-1 (B U)  (eqn:Rasp)."""
    BU = U if B is None else B @ U
    Q = np.zeros_like(BU)
    for sk, Yk in zip(sigma, solve_nodes(lus, BU)):
        Q += sk * Yk
    return Q


def filter_left(lus, sigma, B, V):
    """B^-H rho(M)^H B^H V = sum_k conj(sigma_k) (phi_k B - A)^-H (B^H V)  (eqn:quadf_surMconj)."""
    BhV = V if B is None else B.conj().T @ V
    P = np.zeros_like(BhV)
    for sk, Yk in zip(sigma, solve_nodes(lus, BhV, conj_trans=True)):
        P += np.conj(sk) * Yk
    return P


# ---------------------------------------------------------------------------
# residuals, candidates, stopping
# ---------------------------------------------------------------------------

def residuals(A, B, lam, X):
    """Per column: paper form ||A x - lam B x|| / ||x||, and relative form
    ||A x - lam B x|| / (|lam| ||B x||)."""
    AX = A @ X
    BX = X if B is None else B @ X
    R = AX - BX * lam[None, :]
    rn = np.linalg.norm(R, axis=0)
    xn = np.linalg.norm(X, axis=0)
    bxn = np.linalg.norm(BX, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        paper = rn / xn
        rel = rn / (np.abs(lam) * bxn)
    return paper, rel


def left_residuals(A, B, lam, Y):
    """Per column: ||(A - lam B)^H y|| / (|lam| ||B^H y||)."""
    AhY = A.conj().T @ Y
    BhY = Y if B is None else B.conj().T @ Y
    R = AhY - BhY * np.conj(lam)[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.linalg.norm(R, axis=0) / (np.abs(lam) * np.linalg.norm(BhY, axis=0))


@dataclasses.dataclass
class FeastResult:
    lam: np.ndarray               # candidate eigenvalues (inside, residual <= 1e-4)
    X: np.ndarray                 # their right eigenvectors, unit 2-norm columns
    resid: np.ndarray             # relative residuals of the candidates
    resid_paper: np.ndarray       # paper-form residuals of the candidates
    iters: int
    converged: bool
    history: List[dict]
    ritz: np.ndarray              # all p Ritz values of the last iteration
    Y: Optional[np.ndarray] = None  # left eigenvectors (Bi-FEAST)
    resid_left: Optional[np.ndarray] = None

    @property
    def m(self):
        return len(self.lam)


def _domain(c, R, a, pieces):
    """Membership test of the search domain: the ellipse (c, R, a), or the glued contour's pieces
    (Section 5.4) when given."""
    if pieces:
        return lambda mu: inside_glued(mu, pieces)
    return lambda mu: inside(mu, c, R, a)


def _nodes(c, R, a, rule, q, pieces):
    return glued_nodes_and_weights(pieces, rule, q) if pieces else nodes_and_weights(c, R, a, rule, q)


def _select(lam, paper, rel, dom):
    finite = np.isfinite(lam) & np.isfinite(paper)
    return finite & dom(np.where(finite, lam, 0)) & (paper <= CANDIDATE_RESIDUAL)


def _converged(cand, rel, count, prev_count, n_inside, prev_inside, tol):
    """Stop when the candidate count repeats and every candidate has relative residual <= tol.
    An empty candidate set only counts once no Ritz value at all lies inside, twice in a row
    (otherwise early iterations, whose Ritz pairs are not yet candidates, would stop)."""
    if prev_count is None or count != prev_count:
        return False
    if count == 0:
        return n_inside == 0 and prev_inside == 0
    return bool(np.all(rel[cand] <= tol))


def _n_inside(lam, dom):
    finite = np.isfinite(lam)
    return int(np.count_nonzero(finite & dom(np.where(finite, lam, 0))))


def orthonormalize(Q):
    """Thin QR: an orthonormal basis of span(Q) (Householder, LAPACK zgeqrf)."""
    Qo, _ = np.linalg.qr(Q, mode="reduced")
    return Qo


def rfeast(A, B, c, R, a, q, U0, rule=RULE_TRAPEZOID, tol=1e-10, max_iter=30, lus=None, pieces=None):
    """Algorithm R-FEAST (Section 4).

    Repeat: U^ = rho(M) U_(k-1); orthonormalise U^; A^ = U^H A U^,
    B^ = U^H B U^; solve A^ W = B^ W Lambda^ (QZ); U_(k) = U^ W.
    The domain is the ellipse (c, R, a), or the glued contour `pieces` (Section 5.4)."""
    n = A.shape[0]
    z, sigma = _nodes(c, R, a, rule, q, pieces)
    dom = _domain(c, R, a, pieces)
    if lus is None:
        lus = factor_nodes(A, B, z)
    Bm = _B(B, n)
    U = np.array(U0, dtype=np.complex128)
    history = []
    prev_count = prev_inside = prev_trace = None
    for it in range(1, max_iter + 1):
        Uh = orthonormalize(filter_right(lus, sigma, B, U))
        Ah = Uh.conj().T @ (A @ Uh)
        Bh = Uh.conj().T @ (Bm @ Uh)
        lam, W = scipy.linalg.eig(Ah, Bh)
        X = Uh @ W
        X = X / np.linalg.norm(X, axis=0)[None, :]
        paper, rel = residuals(A, B, lam, X)
        cand = _select(lam, paper, rel, dom)
        count = int(cand.sum())
        trace = complex(lam[cand].sum())
        history.append(dict(iter=it, count=count, trace=trace,
                            trace_change=None if prev_trace is None else abs(trace - prev_trace),
                            res_paper=float(paper[cand].max()) if count else float("nan"),
                            res_rel=float(rel[cand].max()) if count else float("nan")))
        n_in = _n_inside(lam, dom)
        done = _converged(cand, rel, count, prev_count, n_in, prev_inside, tol)
        prev_count, prev_inside, prev_trace = count, n_in, trace
        if done or it == max_iter:
            return FeastResult(lam[cand], X[:, cand], rel[cand], paper[cand], it, done, history, lam)
        U = X


def lfeast(A, B, c, R, a, q, V0, rule=RULE_TRAPEZOID, tol=1e-10, max_iter=30, lus=None, pieces=None):
    """The left-projector variant of R-FEAST (Section 4 notes that it works the same way): the basis
    is filtered by the left filter of eqn:quadf_surMconj, V^ = B^-H rho(M)^H B^H V, and Rayleigh-Ritz
    uses the adjoint pencil, A^ = V^H A^H V^, B^ = V^H B^H V^, whose eigenvalues mu are the conjugates
    of the eigenvalues of (A, B): lambda = conj(mu), left eigenvectors y = V^ W with
    A^H y = conj(lambda) B^H y.  Candidates and stopping as in R-FEAST, with the residual of the left
    pairs."""
    n = A.shape[0]
    z, sigma = _nodes(c, R, a, rule, q, pieces)
    dom = _domain(c, R, a, pieces)
    if lus is None:
        lus = factor_nodes(A, B, z)
    Bm = _B(B, n)
    V = np.array(V0, dtype=np.complex128)
    history = []
    prev_count = prev_inside = prev_trace = None
    for it in range(1, max_iter + 1):
        Vh = orthonormalize(filter_left(lus, sigma, B, V))
        Ah = Vh.conj().T @ (A.conj().T @ Vh)
        Bh = Vh.conj().T @ (Bm.conj().T @ Vh)
        mu, W = scipy.linalg.eig(Ah, Bh)
        lam = np.conj(mu)
        Y = Vh @ W
        Y = Y / np.linalg.norm(Y, axis=0)[None, :]
        # residuals of the left pairs: those of the adjoint pencil at mu
        paper, rel = residuals(A.conj().T, Bm.conj().T, mu, Y)
        cand = _select(lam, paper, rel, dom)
        count = int(cand.sum())
        trace = complex(lam[cand].sum())
        history.append(dict(iter=it, count=count, trace=trace,
                            trace_change=None if prev_trace is None else abs(trace - prev_trace),
                            res_paper=float(paper[cand].max()) if count else float("nan"),
                            res_rel=float(rel[cand].max()) if count else float("nan")))
        n_in = _n_inside(lam, dom)
        done = _converged(cand, rel, count, prev_count, n_in, prev_inside, tol)
        prev_count, prev_inside, prev_trace = count, n_in, trace
        if done or it == max_iter:
            return FeastResult(lam[cand], Y[:, cand], rel[cand], paper[cand], it, done, history, lam)
        V = Y


def biorthogonal_start(B, U0):
    """V0 with V0^H B U0 = I: V0 = B U0 (U0^H B^H B U0)^-1."""
    BU = U0 if B is None else B @ U0
    G = BU.conj().T @ BU
    return BU @ np.linalg.inv(G)


def bifeast(A, B, c, R, a, q, U0, rule=RULE_TRAPEZOID, tol=1e-10, max_iter=30, lus=None, V0=None, pieces=None):
    """Algorithm Bi-FEAST (Section 4).

    Repeat: U^ = rho(M) U, V^ = B^-H rho(M)^H B^H V; orthonormalise both;
    A^ = V^H A U^, B^ = V^H B U^; solve the two-sided reduced problem for
    Lambda^, right vectors W and left vectors Z with Z^H B^ W = I;
    U = U^ W, V = V^ Z, then restore V^H B U = I.
    The domain is the ellipse (c, R, a), or the glued contour `pieces` (Section 5.4)."""
    n = A.shape[0]
    z, sigma = _nodes(c, R, a, rule, q, pieces)
    dom = _domain(c, R, a, pieces)
    if lus is None:
        lus = factor_nodes(A, B, z)
    Bm = _B(B, n)
    U = np.array(U0, dtype=np.complex128)
    V = biorthogonal_start(B, U) if V0 is None else np.array(V0, dtype=np.complex128)
    history = []
    prev_count = prev_inside = prev_trace = None
    for it in range(1, max_iter + 1):
        Uh = orthonormalize(filter_right(lus, sigma, B, U))
        Vh = orthonormalize(filter_left(lus, sigma, B, V))
        Ah = Vh.conj().T @ (A @ Uh)
        Bh = Vh.conj().T @ (Bm @ Uh)
        lam, Zl, Wr = scipy.linalg.eig(Ah, Bh, left=True, right=True)
        d = np.einsum("ij,ik,kj->j", Zl.conj(), Bh, Wr)       # diag(Z^H B^ W)
        Zl = Zl / np.conj(d)[None, :]
        U = Uh @ Wr
        V = Vh @ Zl
        G = (Bm @ U).conj().T @ V                            # U^H B^H V
        V = V @ np.linalg.inv(G)
        X = U / np.linalg.norm(U, axis=0)[None, :]
        Yl = V / np.linalg.norm(V, axis=0)[None, :]
        paper, rel = residuals(A, B, lam, X)
        rel_left = left_residuals(A, B, lam, Yl)
        cand = _select(lam, paper, rel, dom)
        count = int(cand.sum())
        trace = complex(lam[cand].sum())
        history.append(dict(iter=it, count=count, trace=trace,
                            trace_change=None if prev_trace is None else abs(trace - prev_trace),
                            res_paper=float(paper[cand].max()) if count else float("nan"),
                            res_rel=float(rel[cand].max()) if count else float("nan")))
        n_in = _n_inside(lam, dom)
        done = _converged(cand, rel, count, prev_count, n_in, prev_inside, tol)
        prev_count, prev_inside, prev_trace = count, n_in, trace
        if done or it == max_iter:
            return FeastResult(lam[cand], X[:, cand], rel[cand], paper[cand], it, done, history, lam,
                               Y=Yl[:, cand], resid_left=rel_left[cand])


# ---------------------------------------------------------------------------
# mixed-precision references (not in the paper; the precision is never stated there)
# ---------------------------------------------------------------------------

U64 = np.finfo(np.float64).eps / 2


def refinement_threshold(T, Y, rhs, ir_tol=None):
    """Stop when ||rhs - T Y||_F <= tol (||T||_1 ||Y||_F + ||rhs||_F), tol = 8 sqrt(n) u64 by default."""
    n = T.shape[0]
    if ir_tol is None:
        ir_tol = 8.0 * np.sqrt(n) * U64
    return ir_tol * (np.linalg.norm(T, 1) * np.linalg.norm(Y) + np.linalg.norm(rhs))


def solve_refined(T, rhs, low_dtype=np.complex64, ir_max=10, ir_tol=None, factor=None):
    """Low-precision LU of T, FP64 iterative refinement of T Y = rhs.

    Y_0 = solve_low(rhs); repeat R = rhs - T Y (FP64), Y += solve_low(R) until
    ||R|| is below the threshold, or stops halving, or ir_max sweeps.  factor(T) may supply the
    low-precision factorisation in lu_factor layout (default: LAPACK in low_dtype).
    Returns (Y, sweeps, residual norms)."""
    lu = factor(T) if factor is not None else scipy.linalg.lu_factor(T.astype(low_dtype))

    def solve_low(b):
        return scipy.linalg.lu_solve(lu, b.astype(low_dtype)).astype(np.complex128)

    Y = solve_low(rhs)
    norms = []
    sweeps = 0
    for _ in range(ir_max):
        Rk = rhs - T @ Y
        rn = float(np.linalg.norm(Rk))
        norms.append(rn)
        if rn <= refinement_threshold(T, Y, rhs, ir_tol):
            break
        if len(norms) > 1 and rn > 0.5 * norms[-2]:
            break
        Y = Y + solve_low(Rk)
        sweeps += 1
    return Y, sweeps, norms
