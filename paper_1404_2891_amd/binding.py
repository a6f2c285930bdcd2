"""ctypes binding of libfeast_mi355x.so (declared in include/feast_mi355x.h).

Argument marshalling only: every step of the method runs in the HIP library.  PyTorch is used
for device memory (the workspace and the matrices) and for the current HIP stream.  Matrices
are complex128 torch tensors in column-major layout (``t.stride(0) == 1``); use
``to_device(array)`` to upload a NumPy array that way.

If the library has not been built, importing works but every call raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

from . import build as _build

FEAST_OK = 0
FEAST_ENOCONV = 1
FEAST_ERANK = 2
FEAST_EIR = 3
FEAST_EDEVICE = 4
FEAST_EWORKSPACE = 5
FEAST_EREDUCED = 6
FEAST_EUNSUPPORTED = 7
FEAST_ESINGULAR = 1000

RULES = {"trapezoid": 0, "gauss-legendre": 1}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16": 2}
VARIANTS = {"R": 0, "Bi": 1, "L": 2}
BATCH_LAUNCH = {"grouped": 0, "streams": 1}

EXPORTED = [
    "feast_default_options", "feast_contour_nodes", "feast_contour_inside", "feast_workspace_size", "feast_setup",
    "feast_filter", "feast_node_solve", "feast_iterate", "feast_reduced_eig", "feast_destroy",
    "feast_strerror", "feast_timing_read", "feast_timing_reset",
    "feast_batch_workspace_size", "feast_batch_setup", "feast_batch_member", "feast_batch_iterate",
    "feast_batch_factor_ms", "feast_batch_destroy", "feast_batch_trace_estimates", "feast_partition_grid",
    "feast_probe_features", "feast_mlp_param_count", "feast_mlp_workspace_size", "feast_mlp_setup",
    "feast_mlp_fit_standardization", "feast_mlp_forward", "feast_mlp_gradients", "feast_mlp_train_step",
    "feast_mlp_get_params", "feast_m0_from_estimate", "feast_mlp_destroy",
    "feast_autotune_workspace_size", "feast_autotune", "feast_set_panel_rows",
    "feast_filter_shifted", "feast_estimate_m0", "feast_batch_timing_read",
    "feast_mlp_noalloc_max_elems", "feast_mlp_forward_noalloc", "feast_set_m0", "feast_batch_probe_features",
    "feast_autotune_tiles_workspace_size", "feast_autotune_tiles", "feast_set_update_tile",
]


class Piece(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y1", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("kind", ctypes.c_int)]


class Contour(ctypes.Structure):
    _fields_ = [("c_re", ctypes.c_double), ("c_im", ctypes.c_double), ("radius", ctypes.c_double),
                ("aspect", ctypes.c_double), ("q", ctypes.c_int), ("rule", ctypes.c_int),
                ("npieces", ctypes.c_int), ("pieces", ctypes.POINTER(Piece))]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("variant", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("tol", ctypes.c_double), ("candidate_tol", ctypes.c_double), ("ir_max", ctypes.c_int),
                ("ir_tol", ctypes.c_double), ("timing", ctypes.c_int), ("rank_check", ctypes.c_int),
                ("pivoting", ctypes.c_int), ("conj_nodes", ctypes.c_int), ("batch_launch", ctypes.c_int),
                ("host_ortho", ctypes.c_int), ("split_update", ctypes.c_int)]


class PhaseTime(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("flops", ctypes.c_double), ("launches", ctypes.c_long)]


PHASES = ["lu_update", "lu_panel", "lu_other", "solve", "refine", "rayleigh_ritz", "host_reduced_eig",
          "host_cholesky", "host_driver", "host_wait"]


class Result(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("lambda_", ctypes.c_void_p), ("resid", ctypes.c_void_p),
                ("X", ctypes.c_void_p), ("ldx", ctypes.c_int),
                ("Y", ctypes.c_void_p), ("ldy", ctypes.c_int), ("history", ctypes.c_void_p),
                ("ir_sweeps", ctypes.c_int), ("escalated", ctypes.c_int), ("rank", ctypes.c_int)]


class FeastError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} (code {code})")


_lib = None


def library_path() -> str:
    return _build.lib_path()


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_1404_2891_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(path)
        vp, ip, i, d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double
        L.feast_default_options.argtypes = [ctypes.POINTER(Options)]
        L.feast_default_options.restype = None
        L.feast_contour_nodes.argtypes = [ctypes.POINTER(Contour), vp, vp]
        L.feast_contour_nodes.restype = i
        L.feast_contour_inside.argtypes = [ctypes.POINTER(Contour), i, vp, vp]
        L.feast_contour_inside.restype = i
        L.feast_workspace_size.argtypes = [i, i, ctypes.POINTER(Contour), ctypes.POINTER(Options), i,
                                           ctypes.POINTER(ctypes.c_size_t)]
        L.feast_workspace_size.restype = i
        L.feast_setup.argtypes = [ctypes.POINTER(vp), i, vp, i, vp, i, ctypes.POINTER(Contour), i,
                                  ctypes.POINTER(Options), vp, ctypes.c_size_t, vp]
        L.feast_setup.restype = i
        L.feast_filter.argtypes = [vp, i, i, vp, i, vp, i]
        L.feast_filter.restype = i
        L.feast_filter_shifted.argtypes = [vp, i, i, vp, i, vp, vp, i]
        L.feast_filter_shifted.restype = i
        L.feast_estimate_m0.argtypes = [vp, vp, vp, i, i, ctypes.POINTER(i), ctypes.POINTER(d)]
        L.feast_estimate_m0.restype = i
        L.feast_node_solve.argtypes = [vp, i, i, i, vp, i, vp, i]
        L.feast_node_solve.restype = i
        L.feast_iterate.argtypes = [vp, vp, i, ctypes.POINTER(Result)]
        L.feast_iterate.restype = i
        L.feast_reduced_eig.argtypes = [i, vp, vp, vp, vp, vp]
        L.feast_reduced_eig.restype = i
        L.feast_destroy.argtypes = [vp]
        L.feast_destroy.restype = None
        L.feast_timing_read.argtypes = [vp, i, ctypes.POINTER(PhaseTime)]
        L.feast_timing_read.restype = i
        L.feast_timing_reset.argtypes = [vp]
        L.feast_timing_reset.restype = i
        L.feast_strerror.argtypes = [i]
        L.feast_strerror.restype = ctypes.c_char_p
        L.feast_batch_workspace_size.argtypes = [i, vp, vp, vp, ctypes.POINTER(Options), vp,
                                                 ctypes.POINTER(ctypes.c_size_t)]
        L.feast_batch_workspace_size.restype = i
        L.feast_batch_setup.argtypes = [ctypes.POINTER(vp), i, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Options),
                                        vp, ctypes.c_size_t, vp, vp]
        L.feast_batch_setup.restype = i
        L.feast_batch_member.argtypes = [vp, i]
        L.feast_batch_member.restype = vp
        L.feast_batch_iterate.argtypes = [vp, vp, vp, vp, vp]
        L.feast_batch_iterate.restype = i
        L.feast_batch_timing_read.argtypes = [vp, i, ctypes.POINTER(PhaseTime)]
        L.feast_batch_timing_read.restype = i
        L.feast_batch_factor_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.feast_batch_factor_ms.restype = i
        L.feast_batch_trace_estimates.argtypes = [vp, vp, i, i, vp]
        L.feast_batch_trace_estimates.restype = i
        L.feast_partition_grid.argtypes = [i, i, vp, ctypes.c_double, i, ctypes.POINTER(ctypes.c_int), vp, vp]
        L.feast_partition_grid.restype = i
        L.feast_batch_destroy.argtypes = [vp]
        L.feast_batch_destroy.restype = None
        L.feast_probe_features.argtypes = [vp, vp, i, i, vp]
        L.feast_probe_features.restype = i
        L.feast_mlp_param_count.argtypes = [i, i]
        L.feast_mlp_param_count.restype = ctypes.c_long
        L.feast_mlp_workspace_size.argtypes = [i, i, i, ctypes.POINTER(ctypes.c_size_t)]
        L.feast_mlp_workspace_size.restype = i
        L.feast_mlp_setup.argtypes = [ctypes.POINTER(vp), i, i, i, i, vp, vp, ctypes.c_size_t, vp]
        L.feast_mlp_setup.restype = i
        L.feast_mlp_fit_standardization.argtypes = [vp, vp, i]
        L.feast_mlp_fit_standardization.restype = i
        L.feast_mlp_forward.argtypes = [vp, vp, i, vp]
        L.feast_mlp_forward.restype = i
        L.feast_mlp_gradients.argtypes = [vp, vp, vp, i, vp, ctypes.POINTER(d)]
        L.feast_mlp_gradients.restype = i
        L.feast_mlp_train_step.argtypes = [vp, vp, vp, i, d, d, d, d, ctypes.POINTER(d)]
        L.feast_mlp_train_step.restype = i
        L.feast_mlp_get_params.argtypes = [vp, vp]
        L.feast_mlp_get_params.restype = i
        L.feast_m0_from_estimate.argtypes = [d]
        L.feast_m0_from_estimate.restype = i
        L.feast_mlp_destroy.argtypes = [vp]
        L.feast_mlp_destroy.restype = None
        L.feast_autotune_tiles_workspace_size.argtypes = [i, i, ctypes.POINTER(ctypes.c_size_t)]
        L.feast_autotune_tiles_workspace_size.restype = i
        L.feast_autotune_tiles.argtypes = [i, i, vp, ctypes.c_size_t, vp, vp, vp]
        L.feast_autotune_tiles.restype = i
        L.feast_set_update_tile.argtypes = [i, i, i]
        L.feast_set_update_tile.restype = i
        L.feast_batch_probe_features.argtypes = [vp, vp, i, i, vp]
        L.feast_batch_probe_features.restype = i
        L.feast_set_m0.argtypes = [vp, i]
        L.feast_set_m0.restype = i
        L.feast_mlp_noalloc_max_elems.argtypes = []
        L.feast_mlp_noalloc_max_elems.restype = ctypes.c_long
        L.feast_mlp_forward_noalloc.argtypes = [i, i, i, vp, vp, vp, vp, i, vp, vp]
        L.feast_mlp_forward_noalloc.restype = i
        L.feast_autotune_workspace_size.argtypes = [i, i, ctypes.POINTER(ctypes.c_size_t)]
        L.feast_autotune_workspace_size.restype = i
        L.feast_autotune.argtypes = [i, i, vp, ctypes.c_size_t, vp, ctypes.c_char_p, ctypes.POINTER(i), vp]
        L.feast_autotune.restype = i
        L.feast_set_panel_rows.argtypes = [i, i, i]
        L.feast_set_panel_rows.restype = i
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().feast_strerror(code).decode()


def _check(code: int, what: str, ok=(FEAST_OK,)):
    if code not in ok:
        raise FeastError(code, what)
    return code


PIECE_KINDS = {"line": 0, "arc": 1}


def make_pieces(pieces):
    """ctypes array of a glued contour's pieces: ("line", start, end) or ("arc", start, end, center)
    with complex points; an arc runs counterclockwise about its center."""
    arr = (Piece * len(pieces))()
    for P, pc in zip(arr, pieces):
        kind, a, b = pc[0], complex(pc[1]), complex(pc[2])
        c = complex(pc[3]) if kind == "arc" else 0j
        P.x0, P.y0, P.x1, P.y1, P.cx, P.cy = a.real, a.imag, b.real, b.imag, c.real, c.imag
        P.kind = PIECE_KINDS[kind]
    return arr


def polygon(vertices):
    """Pieces of the polygon through the given vertices (counterclockwise order), closed."""
    v = [complex(x) for x in vertices]
    return [("line", v[i], v[(i + 1) % len(v)]) for i in range(len(v))]


def make_contour(center=0j, radius=1.0, aspect=1.0, q=16, rule="trapezoid", pieces=None) -> Contour:
    """The ellipse about center with semi-axes radius and aspect * radius, or, when pieces is given,
    the glued contour of those pieces (center, radius and aspect then unused)."""
    center = complex(center)
    C = Contour(center.real, center.imag, float(radius), float(aspect), int(q), RULES[rule], 0, None)
    if pieces:
        C.npieces = len(pieces)
        C.pieces = make_pieces(pieces)   # ctypes keeps the array alive with the structure
    return C


PIVOTING = {"partial": 0, "tournament": 1}
CONJ_NODES = {"none": 0, "real": 1, "hermitian": 2}


def make_options(precision="fp64", variant="R", max_iter=30, tol=1e-10, candidate_tol=1e-4, ir_max=10,
                 ir_tol=0.0, timing=False, rank_check=False, pivoting="tournament", conj_nodes="none",
                 batch_launch="grouped", host_ortho=False, split_update=True) -> Options:
    o = Options()
    lib().feast_default_options(ctypes.byref(o))
    o.precision = PRECISIONS[precision]
    o.variant = VARIANTS[variant]
    o.max_iter = int(max_iter)
    o.tol = float(tol)
    o.candidate_tol = float(candidate_tol)
    o.ir_max = int(ir_max)
    o.ir_tol = float(ir_tol)
    o.timing = int(bool(timing))
    o.rank_check = int(bool(rank_check))
    o.pivoting = PIVOTING[pivoting]
    o.conj_nodes = CONJ_NODES[conj_nodes]
    o.batch_launch = BATCH_LAUNCH[batch_launch]
    o.host_ortho = int(bool(host_ortho))
    o.split_update = int(bool(split_update))
    return o


def contour_nodes(center=0j, radius=1.0, aspect=1.0, q=16, rule="trapezoid", pieces=None):
    """(z, sigma) of the filter, computed by the library (host)."""
    C = make_contour(center, radius, aspect, q, rule, pieces)
    z = np.zeros(q, dtype=np.complex128)
    s = np.zeros(q, dtype=np.complex128)
    _check(lib().feast_contour_nodes(ctypes.byref(C), z.ctypes.data, s.ctypes.data), "feast_contour_nodes")
    return z, s


def contour_inside(lam, center=0j, radius=1.0, aspect=1.0, q=None, rule="trapezoid", pieces=None):
    """Boolean array: which of the points lam the library counts as inside the contour (host).  The
    node count only has to be valid for the contour (default: two nodes per piece, or 16)."""
    q = (2 * len(pieces) if pieces else 16) if q is None else q
    C = make_contour(center, radius, aspect, q, rule, pieces)
    lam = np.ascontiguousarray(np.atleast_1d(lam), dtype=np.complex128)
    out = np.zeros(lam.shape, dtype=np.int32)
    _check(lib().feast_contour_inside(ctypes.byref(C), lam.size, lam.ctypes.data, out.ctypes.data),
           "feast_contour_inside")
    return out.astype(bool)


def reduced_eig(Ah: np.ndarray, Bh: np.ndarray, left: bool = False):
    """Host reduced eigensolver of the library: (lam, W[, Z])."""
    p = Ah.shape[0]
    Ah = np.asfortranarray(Ah, dtype=np.complex128)
    Bh = np.asfortranarray(Bh, dtype=np.complex128)
    lam = np.zeros(p, dtype=np.complex128)
    W = np.zeros((p, p), dtype=np.complex128, order="F")
    Z = np.zeros((p, p), dtype=np.complex128, order="F") if left else None
    _check(lib().feast_reduced_eig(p, Ah.ctypes.data, Bh.ctypes.data, lam.ctypes.data, W.ctypes.data,
                                   Z.ctypes.data if left else None), "feast_reduced_eig")
    return (lam, W, Z) if left else (lam, W)


def workspace_size(n, m0, contour: Contour, options: Options, has_B: bool) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().feast_workspace_size(n, m0, ctypes.byref(contour), ctypes.byref(options), int(has_B),
                                      ctypes.byref(out)), "feast_workspace_size")
    return out.value


# ---------------------------------------------------------------------------
# torch glue
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def to_device(a: np.ndarray, device="cuda"):
    """Upload a complex NumPy array as a column-major complex128 tensor."""
    torch = _torch()
    a = np.asfortranarray(a, dtype=np.complex128)
    t = torch.from_numpy(a)  # strides (1, n) for Fortran order
    return t.to(device)


def empty_cm(n, k, device="cuda"):
    torch = _torch()
    return torch.empty((k, n), dtype=torch.complex128, device=device).T


def _ld(t) -> int:
    if t.dtype != _torch().complex128:
        raise TypeError("expected complex128")
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("expected a column-major 2-D tensor (stride(0) == 1)")
    return max(t.stride(1), t.shape[0])


def _stream():
    return _torch().cuda.current_stream().cuda_stream


@dataclasses.dataclass
class IterateResult:
    lam: np.ndarray          # candidate eigenvalues
    resid: np.ndarray        # their relative residuals
    X: object                # device tensor n x m (candidate right eigenvectors)
    Y: Optional[object]      # device tensor n x m (left eigenvectors, Bi-FEAST)
    iterations: int
    converged: bool
    history: np.ndarray      # iterations x 4: count, max relative residual, trace re, trace im
    code: int
    ritz: np.ndarray         # all m0 Ritz values (candidates first)
    ir_sweeps: int = 0       # refinement sweeps summed over the run
    escalated: bool = False  # FP16 factorisations replaced by FP32 ones
    rank: int = -1           # numerical rank of the first filtered block (rank check)


class Feast:
    """One pencil: node factorisations resident on the device for the life of the object."""

    def __init__(self, A, B, center=0j, radius=1.0, aspect=1.0, q=16, m0=16, rule="trapezoid",
                 precision="fp64", variant="R", max_iter=30, tol=1e-10, candidate_tol=1e-4, ir_max=10, ir_tol=0.0,
                 timing=False, workspace=None, rank_check=False, pivoting="tournament", pieces=None,
                 conj_nodes="none", host_ortho=False, split_update=True):
        torch = _torch()
        self.n = A.shape[0]
        self.m0 = m0
        self.q = q
        self.A, self.B = A, B
        self.contour = make_contour(center, radius, aspect, q, rule, pieces)
        self.options = make_options(precision, variant, max_iter, tol, candidate_tol, ir_max, ir_tol, timing,
                                    rank_check, pivoting, conj_nodes, host_ortho=host_ortho,
                                    split_update=split_update)
        nbytes = workspace_size(self.n, m0, self.contour, self.options, B is not None)
        if workspace is not None:
            if workspace.numel() < nbytes or workspace.data_ptr() % 256:
                raise ValueError("workspace too small or misaligned")
            self.workspace = workspace
        else:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        self._ctx = ctypes.c_void_p(None)
        code = lib().feast_setup(ctypes.byref(self._ctx), self.n, A.data_ptr(), _ld(A),
                                 None if B is None else B.data_ptr(), 0 if B is None else _ld(B),
                                 ctypes.byref(self.contour), m0, ctypes.byref(self.options),
                                 self.workspace.data_ptr(), nbytes, _stream())
        if code != 0:
            self.setup_code = code
            self.close()
            raise FeastError(code, "feast_setup")
        self.setup_code = 0

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().feast_destroy(self._ctx)
        self._ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def filter(self, U, side=0, out=None):
        """Q = rho(M) U (side 0) or the left filter B^-H rho(M)^H B^H U (side 1)."""
        k = U.shape[1]
        Q = empty_cm(self.n, k, U.device) if out is None else out
        code = lib().feast_filter(self._ctx, side, k, U.data_ptr(), _ld(U), Q.data_ptr(), _ld(Q))
        _check(code, "feast_filter")
        return Q

    def filter_shifted(self, U, lam, side=0, out=None):
        """The shifted-residual form of the filter for the block U and shifts lam (feast_filter_shifted):
        U rho(L) + sum_k sigma_k T_k^-1 (E D_k) with E = A U - B U L (side 1: the left twin)."""
        k = U.shape[1]
        lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128).reshape(-1))
        if lam.size != k:
            raise ValueError("one shift per column")
        Q = empty_cm(self.n, k, U.device) if out is None else out
        _check(lib().feast_filter_shifted(self._ctx, side, k, U.data_ptr(), _ld(U), lam.ctypes.data, Q.data_ptr(),
                                          _ld(Q)), "feast_filter_shifted")
        return Q

    def estimate_m0(self, mlp, V):
        """(m0, m_hat): this context's probe features for V, the perceptron's estimate and the
        subspace-size rule, in one call (feast_estimate_m0)."""
        m0 = ctypes.c_int(0)
        m_hat = ctypes.c_double(0.0)
        _check(lib().feast_estimate_m0(self._ctx, mlp._m, V.data_ptr(), _ld(V), V.shape[1], ctypes.byref(m0),
                                       ctypes.byref(m_hat)), "feast_estimate_m0")
        return m0.value, m_hat.value

    def timing(self) -> dict:
        """Per-phase device time (ms), algorithmic flops and launch counts (needs timing=True)."""
        out = {}
        for i, name in enumerate(PHASES):
            t = PhaseTime()
            _check(lib().feast_timing_read(self._ctx, i, ctypes.byref(t)), "feast_timing_read")
            out[name] = dict(ms=t.ms, flops=t.flops, launches=t.launches)
        return out

    def timing_reset(self):
        _check(lib().feast_timing_reset(self._ctx), "feast_timing_reset")

    def node_solve(self, k, R, side=0):
        Y = empty_cm(self.n, R.shape[1], R.device)
        _check(lib().feast_node_solve(self._ctx, k, side, R.shape[1], R.data_ptr(), _ld(R), Y.data_ptr(), _ld(Y)),
               "feast_node_solve")
        return Y

    def iterate(self, U0) -> IterateResult:
        buf = _ResultBuffers(self.n, self.m0, self.options, U0.device)
        code = lib().feast_iterate(self._ctx, U0.data_ptr(), _ld(U0), ctypes.byref(buf.r))
        _check(code, "feast_iterate", ok=(FEAST_OK, FEAST_ENOCONV, FEAST_ERANK))
        return buf.result(code)

    def set_m0(self, m0):
        """Subspace size of later calls (<= the m0 of the setup); the factorisations stay."""
        _check(lib().feast_set_m0(self._ctx, int(m0)), "feast_set_m0")
        self.m0 = int(m0)

    def probe_features(self, V) -> np.ndarray:
        """Stochastic trace features of this context's filter for the probe block V (device)."""
        k = V.shape[1]
        out = np.zeros(2 * k + 3, dtype=np.float32)
        _check(lib().feast_probe_features(self._ctx, V.data_ptr(), _ld(V), k, out.ctypes.data),
               "feast_probe_features")
        return out


class _ResultBuffers:
    """Caller-owned result buffers of one pencil (host arrays and device blocks)."""

    def __init__(self, n, p, options: Options, device):
        self.lam = np.zeros(p, dtype=np.complex128)
        self.resid = np.zeros(p, dtype=np.float64)
        self.hist = np.full((options.max_iter, 4), np.nan)
        self.X = empty_cm(n, p, device)
        self.Y = empty_cm(n, p, device) if options.variant == 1 else None
        r = Result()
        r.lambda_ = self.lam.ctypes.data
        r.resid = self.resid.ctypes.data
        r.X = self.X.data_ptr()
        r.ldx = _ld(self.X)
        r.Y = self.Y.data_ptr() if self.Y is not None else None
        r.ldy = _ld(self.Y) if self.Y is not None else 0
        r.history = self.hist.ctypes.data
        self.r = r

    def result(self, code) -> IterateResult:
        r, m = self.r, self.r.m
        return IterateResult(self.lam[:m].copy(), self.resid[:m].copy(), self.X[:, :m],
                             None if self.Y is None else self.Y[:, :m], r.iterations, bool(r.converged),
                             self.hist[: r.iterations].copy(), code, self.lam.copy(), r.ir_sweeps,
                             bool(r.escalated), r.rank)


def _ptr_array(values, ctype):
    arr = (ctype * len(values))(*values)
    return arr, ctypes.cast(arr, ctypes.c_void_p)


class FeastBatch:
    """Many pencils factored by one graph launch and iterated in lockstep.

    pencils: list of (A, B) device tensors (B may be None); contours: list of (center, radius, aspect)
    tuples or glued-contour piece lists (see make_pieces), or one tuple for all; m0: list or one int.
    All pencils share q, the rule and the options."""

    def __init__(self, pencils, contours=(0j, 1.0, 1.0), m0=16, q=16, rule="trapezoid", precision="fp64",
                 variant="R", max_iter=30, tol=1e-10, candidate_tol=1e-4, ir_max=10, ir_tol=0.0, workspace=None,
                 rank_check=False, pivoting="tournament", timing=False, batch_launch="grouped", host_ortho=False,
                 split_update=True):
        torch = _torch()
        count = len(pencils)
        self.count = count
        self.pencils = pencils
        self.n = [int(A.shape[0]) for A, _ in pencils]
        self.m0 = list(m0) if isinstance(m0, (list, tuple)) else [int(m0)] * count
        if isinstance(contours, tuple) and not isinstance(contours[0], tuple):
            contours = [contours] * count
        self.options = make_options(precision, variant, max_iter, tol, candidate_tol, ir_max, ir_tol, timing,
                                    rank_check, pivoting, batch_launch=batch_launch, host_ortho=host_ortho,
                                    split_update=split_update)
        C = (Contour * count)(*[make_contour(q=q, rule=rule, pieces=e) if isinstance(e, list)
                                else make_contour(e[0], e[1], e[2], q, rule) for e in contours])
        self._C = C
        n_arr, n_p = _ptr_array(self.n, ctypes.c_int)
        m_arr, m_p = _ptr_array(self.m0, ctypes.c_int)
        hb_arr, hb_p = _ptr_array([int(B is not None) for _, B in pencils], ctypes.c_int)
        nbytes = ctypes.c_size_t(0)
        _check(lib().feast_batch_workspace_size(count, n_p, m_p, ctypes.cast(C, ctypes.c_void_p),
                                                ctypes.byref(self.options), hb_p, ctypes.byref(nbytes)),
               "feast_batch_workspace_size")
        nbytes = nbytes.value
        if workspace is not None:
            if workspace.numel() < nbytes or workspace.data_ptr() % 256:
                raise ValueError("workspace too small or misaligned")
            self.workspace = workspace
        else:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=pencils[0][0].device)
        a_arr, a_p = _ptr_array([A.data_ptr() for A, _ in pencils], ctypes.c_void_p)
        lda_arr, lda_p = _ptr_array([_ld(A) for A, _ in pencils], ctypes.c_int)
        b_arr, b_p = _ptr_array([0 if B is None else B.data_ptr() for _, B in pencils], ctypes.c_void_p)
        ldb_arr, ldb_p = _ptr_array([0 if B is None else _ld(B) for _, B in pencils], ctypes.c_int)
        self.info = np.zeros(count, dtype=np.int32)
        self._b = ctypes.c_void_p(None)
        code = lib().feast_batch_setup(ctypes.byref(self._b), count, n_p, a_p, lda_p, b_p, ldb_p,
                                       ctypes.cast(C, ctypes.c_void_p), m_p, ctypes.byref(self.options),
                                       self.workspace.data_ptr(), nbytes, _stream(), self.info.ctypes.data)
        if code != 0:
            self._b = ctypes.c_void_p(None)
            err = FeastError(code, "feast_batch_setup")
            err.info = self.info.copy()
            raise err

    def factor_ms(self) -> float:
        out = ctypes.c_double(0.0)
        _check(lib().feast_batch_factor_ms(self._b, ctypes.byref(out)), "feast_batch_factor_ms")
        return out.value

    def timing(self) -> dict:
        """Per-phase device time (ms), algorithmic flops and launch counts of the batch (timing=True):
        the factorisation phases of the whole set, the iteration's device phases (grouped launches,
        or summed over the members' own launches) and its host phases for the whole batch."""
        out = {}
        for i, name in enumerate(PHASES):
            t = PhaseTime()
            _check(lib().feast_batch_timing_read(self._b, i, ctypes.byref(t)), "feast_batch_timing_read")
            out[name] = dict(ms=t.ms, flops=t.flops, launches=t.launches)
        return out

    def trace_estimates(self, V) -> np.ndarray:
        """Per member, the stochastic estimate of its eigenvalue count from the probe block V."""
        out = np.zeros(self.count, dtype=np.float64)
        _check(lib().feast_batch_trace_estimates(self._b, V.data_ptr(), _ld(V), V.shape[1], out.ctypes.data),
               "feast_batch_trace_estimates")
        return out

    def probe_features(self, V) -> np.ndarray:
        """Probe features of every pencil (rows), their probe filters launched together."""
        k = V.shape[1]
        out = np.zeros((self.count, 2 * k + 3), dtype=np.float32)
        _check(lib().feast_batch_probe_features(self._b, V.data_ptr(), _ld(V), k, out.ctypes.data),
               "feast_batch_probe_features")
        return out

    def member_probe_features(self, i, V) -> np.ndarray:
        c = lib().feast_batch_member(self._b, i)
        if not c:
            raise IndexError(i)
        k = V.shape[1]
        out = np.zeros(2 * k + 3, dtype=np.float32)
        _check(lib().feast_probe_features(c, V.data_ptr(), _ld(V), k, out.ctypes.data), "feast_probe_features")
        return out

    def set_m0(self, i, m0):
        """Subspace size of pencil i's later iterations (<= its m0 at setup); factorisations stay."""
        c = lib().feast_batch_member(self._b, i)
        if not c:
            raise IndexError(i)
        _check(lib().feast_set_m0(c, int(m0)), "feast_set_m0")
        self.m0[i] = int(m0)

    def member_iterate(self, i, U0) -> IterateResult:
        """feast_iterate on pencil i alone (its own stream, ordered after the batch's)."""
        c = lib().feast_batch_member(self._b, i)
        if not c:
            raise IndexError(i)
        buf = _ResultBuffers(self.n[i], self.m0[i], self.options, U0.device)
        code = lib().feast_iterate(c, U0.data_ptr(), _ld(U0), ctypes.byref(buf.r))
        _check(code, "feast_iterate", ok=(FEAST_OK, FEAST_ENOCONV, FEAST_ERANK))
        return buf.result(code)

    def member_filter(self, i, U, side=0):
        """feast_filter on pencil i alone."""
        c = lib().feast_batch_member(self._b, i)
        if not c:
            raise IndexError(i)
        Q = empty_cm(self.n[i], U.shape[1], U.device)
        _check(lib().feast_filter(c, side, U.shape[1], U.data_ptr(), _ld(U), Q.data_ptr(), _ld(Q)), "feast_filter")
        return Q

    def iterate(self, U0s):
        """feast_iterate on every pencil in lockstep; returns (list of IterateResult, member codes).
        A None start block leaves that pencil out (its result is None)."""
        dev = next(U.device for U in U0s if U is not None)
        bufs = [_ResultBuffers(self.n[i], self.m0[i], self.options, dev) if U0s[i] is not None else None
                for i in range(self.count)]
        res = (Result * self.count)(*[b.r if b is not None else Result() for b in bufs])
        u_arr, u_p = _ptr_array([U.data_ptr() if U is not None else 0 for U in U0s], ctypes.c_void_p)
        ld_arr, ld_p = _ptr_array([_ld(U) if U is not None else 0 for U in U0s], ctypes.c_int)
        rcs = np.zeros(self.count, dtype=np.int32)
        code = lib().feast_batch_iterate(self._b, u_p, ld_p, ctypes.cast(res, ctypes.c_void_p), rcs.ctypes.data)
        _check(code, "feast_batch_iterate", ok=(FEAST_OK, FEAST_ENOCONV, FEAST_ERANK))
        out = []
        for i, b in enumerate(bufs):
            if b is None:
                out.append(None)
                continue
            b.r = res[i]
            out.append(b.result(int(rcs[i])))
        return out, rcs

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            lib().feast_batch_destroy(self._b)
        self._b = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def m0_from_estimate(m_hat: float) -> int:
    return int(lib().feast_m0_from_estimate(float(m_hat)))


def partition_grid(counts, target):
    """Tiles (ix0, ix1, iy0, iy1) of whole cells of the grid counts[ix, iy] with about `target`
    eigenvalues each, and their summed counts (feast_partition_grid)."""
    counts = np.ascontiguousarray(counts, dtype=np.float64)
    gx, gy = counts.shape
    nt = ctypes.c_int(0)
    code = lib().feast_partition_grid(gx, gy, counts.ctypes.data, float(target), 0, ctypes.byref(nt), None, None)
    _check(code, "feast_partition_grid", ok=(FEAST_OK, FEAST_EUNSUPPORTED))
    tiles = np.zeros((max(nt.value, 1), 4), dtype=np.int32)
    sums = np.zeros(max(nt.value, 1), dtype=np.float64)
    _check(lib().feast_partition_grid(gx, gy, counts.ctypes.data, float(target), nt.value, ctypes.byref(nt),
                                      tiles.ctypes.data, sums.ctypes.data), "feast_partition_grid")
    return tiles[: nt.value], sums[: nt.value]


def rectangle(x0, x1, y0, y1):
    """Pieces of the axis-aligned rectangle [x0, x1] x [y0, y1], counterclockwise."""
    return polygon([complex(x0, y0), complex(x1, y0), complex(x1, y1), complex(x0, y1)])


def sized_solve(pencils, contours, start, m0_rule=None, cap=128, probes=None, q=16, precision="fp32",
                chunk=512, **kw):
    """Solve many pencils with the subspace size chosen after their factorisation (Section 4 needs
    m0 >= m; the paper checks it with the rank of the filtered block).  In batches of `chunk`
    pencils (one factorisation each, workspace for `cap` columns): m0 of every pencil from
    m0_rule(features, first index) when given, features = the probe features of the batch's own
    filter for the probe block `probes` (feast_batch_probe_features), else m0 = cap; then the
    lockstep iteration with the rank check; pencils that stop with FEAST_ERANK double their m0 (up
    to cap, feast_set_m0) and iterate again on the same factorisations, without the others.
    pencils: list of (A, B) device tensors; contours: list of (center, radius, aspect);
    start(i, m0): the device start block of pencil i.  Returns (results, m0s, restarts, work) with
    work = dict of algorithmic flops: factorisations, probe solves, iterations."""
    results, m0s, restarts = [None] * len(pencils), [0] * len(pencils), 0
    work = dict(factorisations=0.0, probes=0.0, iterations=0.0)
    for i0 in range(0, len(pencils), chunk):
        part = pencils[i0:i0 + chunk]
        b = FeastBatch(part, contours[i0:i0 + chunk], m0=cap, q=q, precision=precision, rank_check=True, **kw)
        work["factorisations"] += sum(q * (8.0 / 3.0) * int(A.shape[0]) ** 3 for A, _ in part)
        if m0_rule is None:
            m0 = [cap] * len(part)
        else:
            feats = b.probe_features(probes)
            work["probes"] += sum(8.0 * int(A.shape[0]) ** 2 * probes.shape[1] * q for A, _ in part)
            m0 = [max(1, min(cap, int(x))) for x in m0_rule(feats, i0)]
            for k in range(len(part)):
                b.set_m0(k, m0[k])
        todo = list(range(len(part)))
        while todo:
            U0s = [None] * len(part)
            for k in todo:
                U0s[k] = start(i0 + k, m0[k])
            res, rcs = b.iterate(U0s)
            nxt = []
            for k in todo:
                r, rc, n = res[k], rcs[k], int(part[k][0].shape[0])
                work["iterations"] += r.iterations * 8.0 * n * n * m0[k] * (q + 2)
                if rc == FEAST_ERANK and m0[k] < cap:
                    m0[k] = min(2 * m0[k], cap)
                    restarts += 1
                    b.set_m0(k, m0[k])
                    nxt.append(k)
                else:
                    results[i0 + k] = r
                    m0s[i0 + k] = m0[k]
            todo = nxt
        b.close()
    return results, m0s, restarts, work


def multi_domain(A, B, region, probes, grid=(8, 8), target=24, q=16, rule="gauss-legendre", probe_q=8,
                 precision="fp32", variant="R", seed=0, **kw):
    """Eigenvalues of (A, B) inside the rectangle region = (x0, x1, y0, y1), found by load-balanced
    tiles: (1) one probe batch over the grid's cells (glued rectangles, probe_q nodes, FP32, no
    refinement) gives per-cell count estimates from the probe block `probes` (device n x s);
    (2) feast_partition_grid merges cells into tiles of about `target` eigenvalues; (3) one batch
    iterates every tile (q nodes each) with m0 from its estimate and a seeded complex Gaussian
    start block.  Returns (tiles as region rectangles, per-tile estimates, per-tile IterateResult,
    member codes)."""
    torch = _torch()
    x0, x1, y0, y1 = (float(v) for v in region)
    gx, gy = grid
    n = int(A.shape[0])
    xs = np.linspace(x0, x1, gx + 1)
    ys = np.linspace(y0, y1, gy + 1)
    cells = [rectangle(xs[i], xs[i + 1], ys[j], ys[j + 1]) for i in range(gx) for j in range(gy)]
    s = probes.shape[1]
    probe = FeastBatch([(A, B)] * len(cells), cells, m0=s, q=probe_q, rule="gauss-legendre",
                       precision="fp32", ir_max=0)
    est = probe.trace_estimates(probes).reshape(gx, gy)
    probe.close()
    tiles, sums = partition_grid(est, target)
    rects = [(xs[t[0]], xs[t[1]], ys[t[2]], ys[t[3]]) for t in tiles]
    m0s = [min(n, m0_from_estimate(v)) for v in sums]
    batch = FeastBatch([(A, B)] * len(rects), [rectangle(*r) for r in rects], m0=m0s, q=q, rule=rule,
                       precision=precision, variant=variant, **kw)
    g = np.random.default_rng(seed)
    U0s = []
    for m0 in m0s:
        U = (g.standard_normal((n, m0)) + 1j * g.standard_normal((n, m0))) / np.sqrt(2.0)
        U0s.append(to_device(np.asfortranarray(U), A.device))
    res, rcs = batch.iterate(U0s)
    batch.close()
    return rects, sums, res, rcs


class MLP:
    """The subspace-size estimator's perceptron on the device (parameters in the oracle's order)."""

    def __init__(self, params: np.ndarray, n_in=19, hidden=256, max_batch=4096, half=True, device="cuda"):
        torch = _torch()
        self.n_in, self.hidden, self.max_batch = n_in, hidden, max_batch
        self.np = int(lib().feast_mlp_param_count(n_in, hidden))
        params = np.ascontiguousarray(params, dtype=np.float32)
        if params.size != self.np:
            raise ValueError(f"expected {self.np} parameters")
        nbytes = ctypes.c_size_t(0)
        _check(lib().feast_mlp_workspace_size(n_in, hidden, max_batch, ctypes.byref(nbytes)), "feast_mlp_workspace_size")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        self._m = ctypes.c_void_p(None)
        _check(lib().feast_mlp_setup(ctypes.byref(self._m), n_in, hidden, max_batch, int(bool(half)),
                                     params.ctypes.data, self.workspace.data_ptr(), nbytes.value, _stream()),
               "feast_mlp_setup")

    @staticmethod
    def _f32(t):
        torch = _torch()
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError("expected a contiguous float32 tensor")
        return t.data_ptr()

    def fit_standardization(self, X):
        _check(lib().feast_mlp_fit_standardization(self._m, self._f32(X), X.shape[0]), "feast_mlp_fit_standardization")

    def forward(self, X):
        torch = _torch()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(lib().feast_mlp_forward(self._m, self._f32(X), X.shape[0], y.data_ptr()), "feast_mlp_forward")
        return y

    def gradients(self, X, t):
        torch = _torch()
        g = torch.empty(self.np, dtype=torch.float32, device=X.device)
        loss = ctypes.c_double(0.0)
        _check(lib().feast_mlp_gradients(self._m, self._f32(X), self._f32(t), X.shape[0], g.data_ptr(),
                                         ctypes.byref(loss)), "feast_mlp_gradients")
        return g, loss.value

    def train_step(self, X, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=False):
        loss = ctypes.c_double(0.0)
        _check(lib().feast_mlp_train_step(self._m, self._f32(X), self._f32(t), X.shape[0], lr, beta1, beta2, eps,
                                          ctypes.byref(loss) if want_loss else None), "feast_mlp_train_step")
        return loss.value if want_loss else None

    def params(self) -> np.ndarray:
        out = np.zeros(self.np, dtype=np.float32)
        _check(lib().feast_mlp_get_params(self._m, out.ctypes.data), "feast_mlp_get_params")
        return out

    def close(self):
        if getattr(self, "_m", None) is not None and self._m.value:
            lib().feast_mlp_destroy(self._m)
        self._m = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward_noalloc(params, X, n_in=19, hidden=256, half=True, x_mean=None, x_scale=None, out=None):
    """The perceptron's forward pass through feast_mlp_forward_noalloc (no workspace; the library's
    static activation scratch).  params, X, x_mean, x_scale: device float32 tensors; returns y."""
    torch = _torch()
    y = out if out is not None else torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    f = MLP._f32
    _check(lib().feast_mlp_forward_noalloc(n_in, hidden, int(bool(half)), f(params),
                                           None if x_mean is None else f(x_mean),
                                           None if x_scale is None else f(x_scale), f(X), X.shape[0], f(y), _stream()),
           "feast_mlp_forward_noalloc")
    return y


def autotune(precision="fp32", q=16, cache_path=None, device="cuda"):
    """Measure the sweeping/multi-workgroup panel crossover for (precision, q); returns
    (single_rows, table of (rows, sweep ms, multi ms))."""
    torch = _torch()
    nbytes = ctypes.c_size_t(0)
    _check(lib().feast_autotune_workspace_size(q, PRECISIONS[precision], ctypes.byref(nbytes)),
           "feast_autotune_workspace_size")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
    rows = ctypes.c_int(0)
    times = np.zeros(30)
    _check(lib().feast_autotune(PRECISIONS[precision], q, ws.data_ptr(), nbytes.value, _stream(),
                                None if cache_path is None else str(cache_path).encode(), ctypes.byref(rows),
                                times.ctypes.data), "feast_autotune")
    return rows.value, times.reshape(10, 3)


TILE_BUCKET_ROWS = [256, 512, 1024, 2048, 4096, None]   # upper row counts of the tile table's buckets
# per precision argument: the split FP16 update of the FP32 mode, the FP32 matrix-core update (named by
# "fp16", see feast_autotune_tiles), the FP64 update
TILE_SHAPES = {"fp32": ["128x64", "64x64", "64x128"], "fp16": ["128x64", "64x64", "64x128"], "fp64": ["64x64", "128x64"]}


def autotune_tiles(precision="fp32", q=16, device="cuda"):
    """Time the trailing update's tile shapes per row bucket and set the library's tile table;
    returns [(bucket upper rows, chosen shape, {shape: TFLOP/s})]."""
    torch = _torch()
    nbytes = ctypes.c_size_t(0)
    _check(lib().feast_autotune_tiles_workspace_size(PRECISIONS[precision], q, ctypes.byref(nbytes)),
           "feast_autotune_tiles_workspace_size")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
    table = np.zeros(6, dtype=np.int32)
    tf = np.zeros(18, dtype=np.float64)
    _check(lib().feast_autotune_tiles(PRECISIONS[precision], q, ws.data_ptr(), nbytes.value, _stream(),
                                      table.ctypes.data, tf.ctypes.data), "feast_autotune_tiles")
    shapes = TILE_SHAPES[precision]
    return [(TILE_BUCKET_ROWS[b], shapes[table[b]], {shapes[t]: float(tf[3 * b + t]) for t in range(len(shapes))})
            for b in range(6)]


def set_update_tile(precision, bucket, shape_index):
    _check(lib().feast_set_update_tile(PRECISIONS[precision], int(bucket), int(shape_index)), "feast_set_update_tile")


def set_panel_rows(precision, q, rows):
    _check(lib().feast_set_panel_rows(PRECISIONS[precision], q, int(rows)), "feast_set_panel_rows")
