"""Jacobi preconditioner M, plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2, the display that follows the algorithm box: with E = I - A_D^{-1} A,

    G = E^j G_0 + sum_{i=0}^{j-1} E^i A_D^{-1} U      (j >= 1)
    G = U                                               (j  = 0)

where A_D is the diagonal part of A and G_0 the initial guess of the inner
iteration (zero in the paper's tests, Sec. 3.3).  The sum is evaluated
term by term exactly as written; it is the closed form of j Jacobi steps.

Reading of "diagonal part": by default the site-block diagonal of A, i.e.
the 12 x 12 clover matrix T(x) (``jacobi_kind='block'``); the point-diagonal
reading diag(T) is available as ``jacobi_kind='point'``.  The two coincide
when c_SW = 0.
"""

from __future__ import annotations

import numpy as np


def jacobi_apply(op, U: np.ndarray, j: int, G0: np.ndarray | None = None) -> np.ndarray:
    """G = M U for an oracle field U (shape (..., 4, 3, L))."""
    if j < 0:
        raise ValueError("j must be >= 0")
    if j == 0:
        return U.copy()

    def E(v):
        return v - op.apply_AD_inv(op.apply_A(v))

    term = op.apply_AD_inv(U)            # i = 0 term: A_D^{-1} U
    acc = term.copy()
    for _ in range(1, j):                # i = 1 .. j-1
        term = E(term)
        acc = acc + term
    if G0 is not None:
        g = G0
        for _ in range(j):
            g = E(g)
        acc = acc + g
    return acc


def jacobi_mat(op, m: np.ndarray, j: int) -> np.ndarray:
    """M applied to an N x L matrix in the oracle's row order."""
    return op.to_matrix(jacobi_apply(op, op.from_matrix(m), j))

