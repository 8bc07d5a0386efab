"""Preconditioned block BiCGGR, plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The iteration is the algorithm box of Sec. 2, taken step by step in the
paper's order and notation:

    X_0 given;  R_0 = B - A X_0;  P_0 = R_0;  choose Rt_0;  F_0 = M R_0;
    V_0 = W_0 = A F_0
    for k = 0, 1, ...:
        (Rt_0^H V_k) alpha_k = Rt_0^H R_k                   (L x L solve)
        zeta_k = Tr[W_k^H R_k] / Tr[W_k^H W_k]
        S_k = P_k - zeta_k V_k;  U_k = S_k alpha_k
        G_k = M U_k;  Y_k = A G_k
        X_{k+1} = X_k + zeta_k F_k + G_k
        R_{k+1} = R_k - zeta_k W_k - Y_k
        F_{k+1} = M R_{k+1};  W_{k+1} = A F_{k+1}
        (Rt_0^H R_k) gamma_k = Rt_0^H R_{k+1} / zeta_k      (L x L solve)
        P_{k+1} = R_{k+1} + U_k gamma_k;  V_{k+1} = W_{k+1} + Y_k gamma_k

Choices of Sec. 3.3: X_0 = 0, Rt_0 = R_0, stop when
max_i ||r_k^(i)||_2 / ||b^(i)||_2 <= eps on the recursive residual.

Readings where the paper is silent:

* The stopping test is made right after R_{k+1} is formed, before F_{k+1}
  and W_{k+1}.  Counting R_0 as one operator application per column, every
  application of M as j and every A as one, a run that stops in its k-th
  iteration then costs exactly 2(j+1)k + 1 applications per column, which is
  the #MVM/L printed in every entry of Table 1.
* L x L solves use LU with partial pivoting; a pivot below 1e-14 times the
  largest entry (or a non-finite matrix) is reported as a breakdown.
* A maximum relative residual above ``diverge_at`` (1e2, the cut-off used for
  the j = 0 runs in Sec. 3.3) stops the run as diverged; no improvement of
  the best residual over ``stagnate_window`` iterations stops it as
  stagnated.
* Inner products: <a, b> = sum conj(a) b, Tr[W^H R] = sum_{n,i} conj(W_ni) R_ni.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


STATUS = ("converged", "not_converged", "breakdown", "diverged", "stagnated", "nan")


def _lu_solve(C: np.ndarray, rhs: np.ndarray):
    """LU solve with partial pivoting; returns (solution, ok)."""
    if not np.all(np.isfinite(C)):
        return None, False
    scale = np.max(np.abs(C))
    if scale == 0.0:
        return None, False
    lu, piv = scipy.linalg.lu_factor(C, check_finite=False)
    if np.min(np.abs(np.diag(lu))) < 1e-14 * scale:
        return None, False
    return scipy.linalg.lu_solve((lu, piv), rhs, check_finite=False), True


def block_bicggr(A, M, B: np.ndarray, tol: float, j: int, X0: np.ndarray | None = None,
                 max_iter: int = 5000, diverge_at: float = 1e2, stagnate_window: int = 200,
                 callback=None, Rt0: np.ndarray | None = None):
    """Solve A X = B (N x L, complex128) with preconditioned block BiCGGR.

    ``A`` and ``M`` are callables on N x L matrices; ``j`` is the number of
    Jacobi steps in ``M`` (used only for the cost count).  ``callback``, if
    given, is called once per iteration after X_{k+1} and R_{k+1} are formed
    with a dict of the iteration's quantities.  ``Rt0`` is the shadow block
    the algorithm of Sec. 2 leaves free; the default is R_0, the choice of
    the paper's experiments (Sec. 3).  Returns (X, info).
    """
    B = np.asarray(B, dtype=np.complex128)
    N, L = B.shape
    bnorm = np.linalg.norm(B, axis=0)
    if np.any(bnorm == 0):
        raise ValueError("zero right-hand side column")
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.complex128)
    mvm = 0
    R = B - A(X)
    mvm += 1
    P = R.copy()
    Rt = R.copy() if Rt0 is None else np.array(Rt0, dtype=np.complex128)
    F = M(R)
    mvm += j
    W = A(F)
    mvm += 1
    V = W.copy()
    hist = []
    info = dict(status="not_converged", iterations=0, history=hist)

    res0 = np.max(np.linalg.norm(R, axis=0) / bnorm)
    hist.append(res0)
    if res0 <= tol:
        info.update(status="converged", mvm_paper=mvm)
        return X, info

    best, best_k = res0, 0
    C_r = Rt.conj().T @ R                    # Rt_0^H R_k
    for k in range(max_iter):
        C_v = Rt.conj().T @ V                # Rt_0^H V_k
        alpha, ok = _lu_solve(C_v, C_r)
        trWW = np.vdot(W, W)
        if not ok or trWW == 0:
            info.update(status="breakdown", iterations=k, mvm_paper=mvm)
            return X, info
        zeta = np.vdot(W, R) / trWW
        S = P - zeta * V
        U = S @ alpha
        G = M(U)
        mvm += j
        Y = A(G)
        mvm += 1
        X = X + zeta * F + G
        Rn = R - zeta * W - Y
        if callback is not None:
            callback(dict(k=k, X=X, R=R, Rn=Rn, W=W, zeta=zeta, alpha=alpha,
                          C_v=C_v, C_r=C_r))
        res = np.max(np.linalg.norm(Rn, axis=0) / bnorm)
        hist.append(res)
        info["iterations"] = k + 1
        if not np.isfinite(res):
            info.update(status="nan", mvm_paper=mvm)
            return X, info
        if res <= tol:
            info.update(status="converged", mvm_paper=mvm)
            return X, info
        if res > diverge_at:
            info.update(status="diverged", mvm_paper=mvm)
            return X, info
        if res < best:
            best, best_k = res, k + 1
        elif k + 1 - best_k >= stagnate_window:
            info.update(status="stagnated", mvm_paper=mvm)
            return X, info
        F = M(Rn)
        mvm += j
        W = A(F)
        mvm += 1
        C_rn = Rt.conj().T @ Rn              # Rt_0^H R_{k+1}
        if zeta == 0:
            info.update(status="breakdown", mvm_paper=mvm)
            return X, info
        gamma, ok = _lu_solve(C_r, C_rn / zeta)
        if not ok:
            info.update(status="breakdown", mvm_paper=mvm)
            return X, info
        P = Rn + U @ gamma
        V = W + Y @ gamma
        R = Rn
        C_r = C_rn
    info.update(status="not_converged", mvm_paper=mvm)
    return X, info


def true_residual(A, B: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Per-column ||b - A x|| / ||b||."""
    return np.linalg.norm(B - A(X), axis=0) / np.linalg.norm(B, axis=0)


def solve_with_restarts(A, M, B, tol, j, max_restarts: int = 3, **kw):
    """Block BiCGGR followed by a true-residual check; restart from the last X
    (new R_0 = B - A X, Rt_0 = R_0) while some column's true residual exceeds tol."""
    X, info = block_bicggr(A, M, B, tol, j, **kw)
    total_iter = info["iterations"]
    total_mvm = info.get("mvm_paper", 0)
    restarts = 0
    tr = true_residual(A, B, X)
    while info["status"] == "converged" and np.max(tr) > tol and restarts < max_restarts:
        restarts += 1
        X, info = block_bicggr(A, M, B, tol, j, X0=X, **kw)
        total_iter += info["iterations"]
        total_mvm += info.get("mvm_paper", 0)
        tr = true_residual(A, B, X)
    if info["status"] == "converged" and np.max(tr) > tol:
        info["status"] = "not_converged"
    info.update(true_residual=tr, restarts=restarts, total_iterations=total_iter,
                total_mvm_paper=total_mvm)
    return X, info
