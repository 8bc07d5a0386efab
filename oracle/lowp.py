"""The operator and the Jacobi preconditioner with low-precision storage,
plain numpy: the reference for the mixed-precision extension.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes in FP64 only.  The extension stores the links, the site
matrices and the spinors of the inner Jacobi preconditioner in FP32 or BF16
and accumulates in FP32.  The reading fixed here (and the storage the
library uses):

* rounding is round-to-nearest-even, FP64 -> FP32 by the float32 cast and
  FP32 -> BF16 by dropping 16 bits after adding the tie-breaking bias;
* links in FP32 and BF16 are stored as their first two rows only, rows 0
  and 1 of kappa U_mu (scaled in FP64, then rounded); the third row is
  rebuilt in float32 as conj(r_0 x r_1) / kappa, which is kappa times the
  third row of an SU(3) matrix (unitary, unit determinant), and is not
  rounded to the storage format;
* what else is stored: T and T^{-1}
  (built and inverted in FP64, then rounded), the input spinor field, and
  in a j-step Jacobi application the right-hand side and the iterates
  G_1 .. G_{j-1}; the final result is returned unrounded;
* arithmetic is float32 (numpy complex64), in whatever order numpy uses.

Functions equal ``dirac.WilsonClover.apply_A`` and ``jacobi.jacobi_apply``
exactly (up to FP64 rounding) when the format is "f64".
"""

from __future__ import annotations

import numpy as np


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (kept in float32), round to nearest, ties to even:
    the 16 low bits of the float32 pattern are dropped after adding 0x7fff plus the lowest
    kept bit.  Finite inputs only."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def store(z: np.ndarray, fmt: str) -> np.ndarray:
    """A complex field as stored in format fmt ("f64", "f32" or "bf16"): complex128 for "f64",
    else complex64 with the real and imaginary parts rounded to float32 and, for "bf16",
    further to bfloat16."""
    if fmt == "f64":
        return np.asarray(z, dtype=np.complex128)
    z = np.asarray(z).astype(np.complex64)
    if fmt == "bf16":
        z = (round_bf16(z.real) + 1j * round_bf16(z.imag)).astype(np.complex64)
    return z


class LowpOperator:
    """The pieces of A with their coefficients stored in fmt: kappa-scaled links, T and T^{-1}
    (taken from an FP64 ``dirac.WilsonClover``), and the hop and site products in the
    arithmetic of that format (float32 unless fmt is "f64")."""

    def __init__(self, op, fmt: str):
        self.op = op
        self.fmt = fmt
        self.links = [store(op.kappa * op.U[mu], fmt) for mu in range(4)]
        if fmt != "f64":
            invk = np.float32(1.0 / op.kappa) if op.kappa != 0 else np.float32(0.0)
            for lk in self.links:
                r0, r1 = lk[..., 0, :], lk[..., 1, :]
                lk[..., 2, :] = np.conj(np.cross(r0, r1)) * invk
        self.T = store(op.T, fmt)
        self.Tinv = store(op.Tinv, fmt)
        cdt = np.complex128 if fmt == "f64" else np.complex64
        self.g = op.g.astype(cdt)
        self.one = np.eye(4, dtype=cdt)

    def khop(self, f):
        """kappa H f with the stored (kappa-scaled) links."""
        op = self.op
        out = np.zeros_like(f)
        for mu in range(4):
            fwd = np.roll(f, -1, axis=3 - mu).copy()
            bwd = np.roll(f, 1, axis=3 - mu).copy()
            if mu == 3 and op.bc_t == 1:
                fwd[-1] *= -1
                bwd[0] *= -1
            Ub = np.roll(self.links[mu], 1, axis=3 - mu)
            uf = np.einsum("...ab,...sbl->...sal", self.links[mu], fwd)
            ub = np.einsum("...ba,...sbl->...sal", np.conj(Ub), bwd)
            out += np.einsum("st,...tal->...sal", self.one - self.g[mu], uf)
            out += np.einsum("st,...tal->...sal", self.one + self.g[mu], ub)
        return out

    def site(self, M, f):
        L = f.shape[-1]
        return (M @ f.reshape(self.op.shape + (12, L))).reshape(self.op.shape + (4, 3, L))


def apply_lowp(op, X: np.ndarray, fmt: str) -> np.ndarray:
    """A X (Sec. 2's operator, the convention of ``dirac``) with X, the links and T stored in
    fmt and float32 arithmetic; returned as complex128."""
    lo = LowpOperator(op, fmt)
    x = store(X, fmt)
    return np.asarray(lo.site(lo.T, x) - lo.khop(x), dtype=np.complex128)


def jacobi_sweeps_lowp(op, U: np.ndarray, j: int, fmt: str) -> np.ndarray:
    """G = M U for the block reading of A_D as j sweeps G_{i+1} = T^{-1} (U + kappa H G_i),
    G_0 = 0 (the recurrence whose closed form is the paper's sum, Sec. 2), with T^{-1}, the
    links, the right-hand side and the iterates G_1 .. G_{j-1} stored in fmt and float32
    arithmetic.  With j = 1 the right-hand side is only converted to FP32 (the single sweep
    reads it once).  The last sweep is returned unrounded (complex128)."""
    if j == 0:
        return np.array(U, dtype=np.complex128)
    lo = LowpOperator(op, fmt)
    rhs = store(U, fmt) if (j > 1 or fmt == "f64") else store(U, "f32")
    G = lo.site(lo.Tinv, rhs)
    for _ in range(1, j):
        G = lo.site(lo.Tinv, rhs + lo.khop(store(G, fmt)))
    return np.asarray(G, dtype=np.complex128)
