"""ctypes binding of the wdsolve C ABI (``include/wdsolve.h``).

Argument marshalling only: every numerical step runs in the HIP library.
The binding refuses to work without the built library; there is no
fallback path.

Device memory is handled with PyTorch tensors (complex128 on a ROCm device):
block vectors are tensors of shape (L, 12, V) -- column i, spin-colour
k = 3*spin + colour, site s -- which is exactly the ABI's N x L column-major
layout with row n = k*V + s.  After ``Context.set_layout("tiled")`` the same
tensors hold the tiled row order n = (s//64)*768 + k*64 + s%64.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_longlong, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwdsolve.so")

WD_OK = 0
WD_EINVAL = -1
WD_ENOMEM = -2
WD_EHIP = -3
WD_ENAN = -4
WD_ESTATE = -5
WD_NOT_CONVERGED = 1
WD_BREAKDOWN = 2
WD_DIVERGED = 3
WD_STAGNATED = 4

WD_F64, WD_F32, WD_BF16 = 0, 1, 2
WD_F64_COEF_F32, WD_F64_COEF_BF16 = 3, 4   # Jacobi only: FP64 iterates, low-precision links and A_D^-1
WD_PRECOND_NONE, WD_PRECOND_JACOBI, WD_PRECOND_LEARNED = 0, 1, 2
WD_LEARNED_INIT_IDENTITY, WD_LEARNED_INIT_NEUMANN = 0, 1
WD_LOSS_ERROR, WD_LOSS_RESIDUAL = 0, 1
LOSS = {"error": WD_LOSS_ERROR, "residual": WD_LOSS_RESIDUAL}
WD_JACOBI_BLOCK, WD_JACOBI_POINT = 0, 1
WD_MAX_L = 16
WD_LAYOUT_STANDARD, WD_LAYOUT_TILED = 0, 1
LAYOUT = {"standard": WD_LAYOUT_STANDARD, "tiled": WD_LAYOUT_TILED}

PREC = {"f64": WD_F64, "f32": WD_F32, "bf16": WD_BF16, "f64c32": WD_F64_COEF_F32, "f64cbf16": WD_F64_COEF_BF16}
STATUS_NAME = {WD_OK: "converged", WD_NOT_CONVERGED: "not_converged", WD_BREAKDOWN: "breakdown",
               WD_DIVERGED: "diverged", WD_STAGNATED: "stagnated", WD_ENAN: "nan"}


class SolveOpts(ctypes.Structure):
    _fields_ = [("j", c_int), ("precond", c_int), ("prec_inner", c_int), ("use_x0", c_int),
                ("max_iter", c_int), ("max_restarts", c_int), ("stagnate_window", c_int),
                ("diverge_at", c_double), ("history", POINTER(c_double)), ("history_len", c_int),
                ("cycle_tol", c_double), ("no_fallback", c_int), ("x_snap", c_void_p), ("snap_count", c_int),
                ("snap_every", c_int), ("gap_history", POINTER(c_double)), ("cond_history", POINTER(c_double)),
                ("cond_limit", c_double), ("no_split", c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", c_int), ("iterations", c_int), ("total_iterations", c_int), ("restarts", c_int),
                ("cycles", c_int), ("fallback", c_int), ("snapshots", c_int),
                ("mvm_paper", c_longlong), ("mvm_actual", c_longlong), ("seconds", c_double),
                ("bytes_alg", c_double),
                ("true_residual", c_double * WD_MAX_L), ("recursive_residual", c_double * WD_MAX_L),
                ("cond_max", c_double), ("splits", c_int), ("min_block", c_int)]


class WDError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


# (name, restype, argtypes) of every exported function
SIGNATURES = [
    ("wd_create", c_int, [POINTER(c_void_p), POINTER(c_int), c_int, c_int, c_void_p]),
    ("wd_destroy", c_int, [c_void_p]),
    ("wd_set_links", c_int, [c_void_p, c_void_p, c_int]),
    ("wd_set_params", c_int, [c_void_p, c_double, c_double, c_int]),
    ("wd_get_clover", c_int, [c_void_p, c_int, c_void_p]),
    ("wd_set_layout", c_int, [c_void_p, c_int]),
    ("wd_apply", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int]),
    ("jacobi_precond", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int]),
    ("bbicggr_solve", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_double, POINTER(SolveOpts),
                              POINTER(SolveInfo)]),
    ("bbicgstab_solve", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_double, POINTER(SolveOpts),
                                POINTER(SolveInfo)]),
    ("wd_hop_repeat", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int]),
    ("wd_block_gram", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    ("wd_small_solve", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    ("wd_block_gram_static", c_int, [c_void_p, c_void_p, c_longlong, c_int, c_void_p, c_void_p]),
    ("wd_set_learned", c_int, [c_void_p, c_void_p]),
    ("wd_learned_init", c_int, [c_void_p, c_int]),
    ("wd_learned_pairs", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    ("wd_get_learned", c_int, [c_void_p, c_void_p]),
    ("wd_learned_apply", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int]),
    ("wd_learned_train", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_double, c_int, c_void_p]),
    ("wd_learned_grad", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    ("wd_strerror", ctypes.c_char_p, [c_int]),
    ("wd_volume", c_longlong, [c_void_p]),
]

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"wdsolve HIP library not found at {path}; build it with "
                          "`python -m paper_0907_3261_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().wd_strerror(code).decode()


def _check(code: int, what: str) -> int:
    if code < 0:
        raise WDError(code, what)
    return code


def _torch():
    import torch
    return torch


def _dptr(t) -> int:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


class Context:
    """One lattice, gauge field and operator; all work on one HIP stream."""

    def __init__(self, dims, bc_t: int = 0, max_L: int = 12, stream=None, device: int = 0):
        torch = _torch()
        lib = load()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.N = 12 * self.V
        self.max_L = int(max_L)
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = c_void_p()
        d = (c_int * 4)(*self.dims)
        with torch.cuda.device(self.device):
            _check(lib.wd_create(ctypes.byref(h), d, int(bc_t), self.max_L, c_void_p(stream.cuda_stream)),
                   "wd_create")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.wd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup
    def set_links(self, U):
        """U: complex128 array/tensor of shape (4, V, 3, 3) (host numpy or device tensor)."""
        torch = _torch()
        if isinstance(U, np.ndarray):
            a = np.ascontiguousarray(U, dtype=np.complex128)
            if a.shape != (4, self.V, 3, 3):
                raise ValueError("links must have shape (4, V, 3, 3)")
            _check(self._lib.wd_set_links(self._h, a.ctypes.data, 0), "wd_set_links")
        else:
            if U.dtype != torch.complex128 or tuple(U.shape) != (4, self.V, 3, 3):
                raise ValueError("links must be complex128 of shape (4, V, 3, 3)")
            _check(self._lib.wd_set_links(self._h, _dptr(U), 1), "wd_set_links")

    def set_params(self, kappa: float, csw: float, jacobi_kind: int = WD_JACOBI_BLOCK):
        _check(self._lib.wd_set_params(self._h, float(kappa), float(csw), int(jacobi_kind)), "wd_set_params")

    def clover(self, which: int = 0) -> np.ndarray:
        """T (which=0) or T^-1 (which=1) as (V, 2, 6, 6) complex128 on the host."""
        out = np.empty((self.V, 2, 6, 6), dtype=np.complex128)
        _check(self._lib.wd_get_clover(self._h, int(which), out.ctypes.data), "wd_get_clover")
        return out

    def set_layout(self, layout: str):
        """Row layout of the block vectors this context reads and writes: "standard"
        (row k*V + s) or "tiled" (row (s//64)*768 + k*64 + s%64); tensors keep the shape
        (L, 12, V) either way."""
        _check(self._lib.wd_set_layout(self._h, LAYOUT[layout]), "wd_set_layout")

    # ---- hot path
    def _block(self, t, L=None):
        torch = _torch()
        if t.dtype != torch.complex128 or t.dim() != 3 or t.shape[1] != 12 or t.shape[2] != self.V:
            raise ValueError("block vectors are complex128 tensors of shape (L, 12, V)")
        if L is not None and t.shape[0] != L:
            raise ValueError("column count mismatch")
        return _dptr(t)

    def _snap_ptr(self, t, L):
        """x_snap: complex128 tensor of shape (n * L, 12, V); n snapshots of L columns."""
        if t is None:
            return None
        torch = _torch()
        if t.dtype != torch.complex128 or t.dim() != 3 or t.shape[1] != 12 or t.shape[2] != self.V or \
                t.shape[0] % L or not t.is_contiguous():
            raise ValueError("x_snap must be a contiguous complex128 tensor of shape (n * L, 12, V)")
        return _dptr(t)

    def empty_block(self, L: int):
        return _torch().empty((L, 12, self.V), dtype=_torch().complex128, device=self.device)

    def apply(self, X, Y=None, prec: str = "f64"):
        L = X.shape[0]
        if Y is None:
            Y = self.empty_block(L)
        _check(self._lib.wd_apply(self._h, self._block(X), self._block(Y, L), L, PREC[prec]), "wd_apply")
        return Y

    def jacobi(self, R, j: int, Z=None, prec: str = "f64"):
        L = R.shape[0]
        if Z is None:
            Z = self.empty_block(L)
        _check(self._lib.jacobi_precond(self._h, self._block(R), self._block(Z, L), L, int(j), PREC[prec]),
               "jacobi_precond")
        return Z

    def solve(self, B, X=None, tol: float = 1e-12, j: int = 0, precond: int | None = None,
              prec_inner: str = "f64", max_iter: int = 0, max_restarts: int = -1, diverge_at: float = 0.0,
              stagnate_window: int = 0, history_len: int = 0, cycle_tol: float = 0.0,
              no_fallback: bool = False, x_snap=None, snap_every: int = 0, gap_history: bool = False,
              cond_history: bool = False, cond_limit: float = 0.0, no_split: bool = False,
              method: str = "bicggr"):
        """Preconditioned block BiCGGR (method "bicggr") or the block BiCGSTAB foil ("bicgstab");
        returns (X, info dict).  X, if given, is the initial guess.  gap_history / cond_history
        ask for the per-iteration residual gap and condition estimate (history_len entries)."""
        L = B.shape[0]
        use_x0 = X is not None
        if X is None:
            X = self.empty_block(L)
        if precond is None:
            precond = WD_PRECOND_JACOBI if j > 0 else WD_PRECOND_NONE
        n_hist = max(history_len, 1)
        hist = (c_double * n_hist)()
        ghist = (c_double * n_hist)()
        chist = (c_double * n_hist)()
        o = SolveOpts(j=int(j), precond=int(precond), prec_inner=PREC[prec_inner], use_x0=int(use_x0),
                      max_iter=int(max_iter), max_restarts=int(max_restarts),
                      stagnate_window=int(stagnate_window), diverge_at=float(diverge_at),
                      history=ctypes.cast(hist, POINTER(c_double)) if history_len else None,
                      history_len=int(history_len), cycle_tol=float(cycle_tol),
                      no_fallback=int(bool(no_fallback)),
                      x_snap=self._snap_ptr(x_snap, L), snap_count=(x_snap.shape[0] // L) if x_snap is not None else 0,
                      snap_every=int(snap_every),
                      gap_history=ctypes.cast(ghist, POINTER(c_double)) if (history_len and gap_history) else None,
                      cond_history=ctypes.cast(chist, POINTER(c_double)) if (history_len and cond_history) else None,
                      cond_limit=float(cond_limit), no_split=int(bool(no_split)))
        info = SolveInfo()
        fn = {"bicggr": self._lib.bbicggr_solve, "bicgstab": self._lib.bbicgstab_solve}[method]
        code = fn(self._h, self._block(B), self._block(X, L), L, float(tol), ctypes.byref(o), ctypes.byref(info))
        if code != WD_ENAN:          # a non-finite residual is an outcome of the solve, reported in info
            _check(code, method)
        d = dict(code=code, status=STATUS_NAME.get(code, str(code)), info_status=info.status,
                 iterations=info.iterations,
                 total_iterations=info.total_iterations, restarts=info.restarts, cycles=info.cycles,
                 fallback=bool(info.fallback), snapshots=info.snapshots,
                 mvm_paper=info.mvm_paper,
                 mvm_actual=info.mvm_actual, seconds=info.seconds, bytes_alg=info.bytes_alg,
                 true_residual=np.array(info.true_residual[:L]),
                 recursive_residual=np.array(info.recursive_residual[:L]),
                 cond_max=info.cond_max, splits=info.splits, min_block=info.min_block)
        if history_len:
            n = min(history_len, info.total_iterations + info.cycles)
            d["history"] = np.array(hist[:n])
            if gap_history:
                d["gap_history"] = np.array(ghist[:n])
            if cond_history:
                d["cond_history"] = np.array(chist[:n])
        return X, d

    def hop_repeat(self, X, Y, nrep: int, mode: int = 0, R=None, prec: str = "f64"):
        """Launch the hopping kernel nrep times back to back (mode 0: A X, 1: Jacobi sweep)."""
        L = X.shape[0]
        r = self._block(R, L) if R is not None else None
        _check(self._lib.wd_hop_repeat(self._h, self._block(X), r, self._block(Y, L), L, int(mode), PREC[prec],
                                       int(nrep)), "wd_hop_repeat")
        return Y

    # ---- learned preconditioner
    def set_learned(self, theta: np.ndarray):
        """theta: complex array (3, 9, 4, 4), stored as complex64."""
        a = np.ascontiguousarray(np.asarray(theta).reshape(3, 9, 4, 4), dtype=np.complex64)
        _check(self._lib.wd_set_learned(self._h, a.ctypes.data), "wd_set_learned")

    def learned_init(self, kind: str = "neumann"):
        """theta := identity (M = 1) or the factored degree-3 Neumann series of (1 - kappa H)^-1."""
        k = {"identity": WD_LEARNED_INIT_IDENTITY, "neumann": WD_LEARNED_INIT_NEUMANN}[kind]
        _check(self._lib.wd_learned_init(self._h, k), "wd_learned_init")

    def learned_pairs(self, B, X, Xsnap):
        """Pairs (Rp, Ep) = (B - A X_k, X - X_k) from the solver's snapshots X_k (Xsnap: (n L, 12, V))."""
        L = B.shape[0]
        n = Xsnap.shape[0] // L
        Rp = _torch().empty_like(Xsnap)
        Ep = _torch().empty_like(Xsnap)
        _check(self._lib.wd_learned_pairs(self._h, self._block(B), self._block(X, L), self._snap_ptr(Xsnap, L),
                                          n, L, _dptr(Rp), _dptr(Ep)), "wd_learned_pairs")
        return Rp, Ep

    def get_learned(self) -> np.ndarray:
        a = np.empty((3, 9, 4, 4), dtype=np.complex64)
        _check(self._lib.wd_get_learned(self._h, a.ctypes.data), "wd_get_learned")
        return a

    def learned_apply(self, R, Z=None, prec: str = "f32"):
        L = R.shape[0]
        if Z is None:
            Z = self.empty_block(L)
        _check(self._lib.wd_learned_apply(self._h, self._block(R), self._block(Z, L), L, PREC[prec]),
               "wd_learned_apply")
        return Z

    def learned_train(self, Rp, Ep, L: int, steps: int, lr: float = 1e-3, loss: str = "error"):
        """Train on pairs (Rp, Ep: device tensors of shape (P, 12, V); Ep may be None for the
        residual loss); returns the loss per step."""
        P = Rp.shape[0]
        hist = np.zeros(max(steps, 1), dtype=np.float32)
        e = self._block(Ep, P) if Ep is not None else None
        _check(self._lib.wd_learned_train(self._h, self._block(Rp), e, P, int(L), int(steps), float(lr), LOSS[loss],
                                          hist.ctypes.data), "wd_learned_train")
        return hist[:steps]

    def learned_grad(self, R, E, loss: str = "error"):
        L = R.shape[0]
        lv = ctypes.c_double()
        G = np.empty((3, 9, 4, 4), dtype=np.complex128)
        e = self._block(E, L) if E is not None else None
        _check(self._lib.wd_learned_grad(self._h, self._block(R), e, L, LOSS[loss], ctypes.byref(lv),
                                         G.ctypes.data), "wd_learned_grad")
        return lv.value, G

    # ---- block kernels
    def gram(self, P, Q):
        torch = _torch()
        L = P.shape[0]
        C = torch.empty((L, L), dtype=torch.complex128, device=self.device)
        _check(self._lib.wd_block_gram(self._h, self._block(P), self._block(Q, L), L, _dptr(C)), "wd_block_gram")
        return C

    def gram_static(self, P, Q):
        """P^H Q through the entry point that allocates nothing (no context workspace)."""
        torch = _torch()
        L = P.shape[0]
        C = torch.empty((L, L), dtype=torch.complex128, device=self.device)
        _check(self._lib.wd_block_gram_static(self._block(P), self._block(Q, L), self.N, L, _dptr(C),
                                              c_void_p(self.stream.cuda_stream)), "wd_block_gram_static")
        return C

    def small_solve(self, M, RHS):
        """Solve M Z = RHS for L x L complex128 device tensors; returns (Z, ok)."""
        torch = _torch()
        L = M.shape[0]
        Z = torch.empty((L, L), dtype=torch.complex128, device=self.device)
        code = _check(self._lib.wd_small_solve(self._h, _dptr(M.contiguous()), _dptr(RHS.contiguous()), L,
                                               _dptr(Z)), "wd_small_solve")
        return Z, code == WD_OK
