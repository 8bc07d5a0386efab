"""Preconditioned block BiCGSTAB, plain numpy FP64: the foil of block BiCGGR.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper motivates BiCGGR by the gap that opens, in BiCGSTAB-type block
methods, between the recursively updated residual R_k and the true residual
B - A X_k (Sec. 1); it does not print BiCGSTAB itself.  The block BiCGSTAB
written here follows the published block version of van der Vorst's method
(Guennouni, Jbilou and Sadok, "A block version of BiCGSTAB for linear
systems with multiple right-hand sides", ETNA 16, 2003), with M applied on
the right as in the paper's BiCGGR box:

    X_0 given;  R_0 = B - A X_0;  P_0 = R_0;  choose Rt_0
    for k = 0, 1, ...:
        Ph_k = M P_k;   V_k = A Ph_k
        (Rt_0^H V_k) alpha_k = Rt_0^H R_k                 (L x L solve)
        S_k = R_k - V_k alpha_k
        Sh_k = M S_k;   T_k = A Sh_k
        omega_k = Tr[T_k^H S_k] / Tr[T_k^H T_k]
        X_{k+1} = X_k + Ph_k alpha_k + omega_k Sh_k
        R_{k+1} = S_k - omega_k T_k
        (Rt_0^H V_k) beta_k = -Rt_0^H T_k                 (L x L solve)
        P_{k+1} = R_{k+1} + (P_k - omega_k V_k) beta_k

The coefficient beta_k is the block form of beta = (rho_{k+1} / rho_k)
(alpha / omega): with Rt_0^H S_k = 0 (which alpha_k enforces),
Rt_0^H R_{k+1} = -omega_k Rt_0^H T_k.  Every iteration applies M twice and
A twice, so a run stopped in its k-th iteration costs 2(j+1)k + 1
applications per column, as block BiCGGR does (the stopping test follows the
R update, as in the BiCGGR oracle).
"""

from __future__ import annotations

import numpy as np

from .bbicggr import _lu_solve


def block_bicgstab(A, M, B: np.ndarray, tol: float, j: int, X0: np.ndarray | None = None,
                   max_iter: int = 5000, diverge_at: float = 1e2, stagnate_window: int = 200,
                   callback=None, Rt0: np.ndarray | None = None):
    """Solve A X = B (N x L, complex128) with preconditioned block BiCGSTAB.

    Same calling convention as ``bbicggr.block_bicggr``: ``A`` and ``M`` are
    callables on N x L matrices, ``j`` only enters the cost count, and
    ``callback`` receives the iteration's quantities after X_{k+1} and
    R_{k+1} are formed.  Returns (X, info)."""
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
    hist = []
    info = dict(status="not_converged", iterations=0, history=hist)
    res0 = np.max(np.linalg.norm(R, axis=0) / bnorm)
    hist.append(res0)
    if res0 <= tol:
        info.update(status="converged", mvm_paper=mvm)
        return X, info
    best, best_k = res0, 0
    for k in range(max_iter):
        Ph = M(P)
        mvm += j
        V = A(Ph)
        mvm += 1
        C_v = Rt.conj().T @ V                    # Rt_0^H V_k
        alpha, ok = _lu_solve(C_v, Rt.conj().T @ R)
        if not ok:
            info.update(status="breakdown", iterations=k, mvm_paper=mvm)
            return X, info
        S = R - V @ alpha
        Sh = M(S)
        mvm += j
        T = A(Sh)
        mvm += 1
        trTT = np.vdot(T, T)
        if trTT == 0:
            info.update(status="breakdown", iterations=k, mvm_paper=mvm)
            return X, info
        omega = np.vdot(T, S) / trTT
        X = X + Ph @ alpha + omega * Sh
        Rn = S - omega * T
        if callback is not None:
            callback(dict(k=k, X=X, Rn=Rn, alpha=alpha, omega=omega, C_v=C_v))
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
        if omega == 0:
            info.update(status="breakdown", mvm_paper=mvm)
            return X, info
        beta, ok = _lu_solve(C_v, -(Rt.conj().T @ T))
        if not ok:
            info.update(status="breakdown", mvm_paper=mvm)
            return X, info
        P = Rn + (P - omega * V) @ beta
        R = Rn
    info.update(status="not_converged", mvm_paper=mvm)
    return X, info
