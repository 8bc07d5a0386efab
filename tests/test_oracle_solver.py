"""Pins of the oracle's Jacobi preconditioner and block BiCGGR.

Facts used: the Jacobi polynomial identity M_j A = I - E^j (dense matrices),
the Neumann series at c_SW = 0, convergence of the inner iteration to A^{-1}
when it contracts, dense LU solutions, the residual-consistency property the
method is built for, the least-squares meaning of zeta, the #MVM count of
Table 1, and forced failure paths.
"""

import os

import numpy as np
import pytest

import wdinputs as wi
from oracle import WilsonClover
from oracle.jacobi import jacobi_apply, jacobi_mat
from oracle.bbicggr import block_bicggr, solve_with_restarts, true_residual

HERE = os.path.dirname(os.path.abspath(__file__))


def _op(dims=(2, 2, 2, 2), kappa=0.12, csw=1.2, seed=5, eps=0.5, kind="block", bc_t=0):
    return WilsonClover(dims, wi.random_links(dims, eps, seed), kappa, csw, bc_t=bc_t, jacobi_kind=kind)


# ---------------------------------------------------------------- Jacobi

@pytest.mark.parametrize("kind", ["block", "point"])
@pytest.mark.parametrize("j", [1, 2, 5])
def test_jacobi_polynomial_identity(kind, j):
    """M_j A v = v - E^j v (j >= 1) with E = I - A_D^{-1} A, A_D the (block or point) diagonal of dense A."""
    op = _op(kind=kind, kappa=0.14)
    A = op.dense()
    N = op.N
    if kind == "block":
        AD = np.zeros_like(A)
        for s in range(op.V):
            AD[12 * s:12 * s + 12, 12 * s:12 * s + 12] = A[12 * s:12 * s + 12, 12 * s:12 * s + 12]
    else:
        AD = np.diag(np.diag(A))
    E = np.eye(N) - np.linalg.solve(AD, A)
    v = op.block_to_mat(wi.gaussian_block(op.V, 3, 7))
    lhs = jacobi_mat(op, A @ v, j)
    rhs = v - np.linalg.matrix_power(E, j) @ v
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(v) < 1e-13


def test_jacobi_j0_is_identity():
    op = _op()
    u = op.from_block(wi.gaussian_block(op.V, 2, 6))
    assert np.array_equal(jacobi_apply(op, u, 0), u)


def test_jacobi_initial_guess_term():
    op = _op(kappa=0.1)
    A = op.dense()
    AD = np.zeros_like(A)
    for s in range(op.V):
        AD[12 * s:12 * s + 12, 12 * s:12 * s + 12] = A[12 * s:12 * s + 12, 12 * s:12 * s + 12]
    E = np.eye(op.N) - np.linalg.solve(AD, A)
    u = op.block_to_mat(wi.gaussian_block(op.V, 2, 8))
    g0 = op.block_to_mat(wi.gaussian_block(op.V, 2, 9))
    got = op.to_matrix(jacobi_apply(op, op.from_matrix(u), 3, G0=op.from_matrix(g0)))
    Ei = [np.linalg.matrix_power(E, i) for i in range(4)]
    want = Ei[3] @ g0 + sum(Ei[i] @ np.linalg.solve(AD, u) for i in range(3))
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13


@pytest.mark.parametrize("kind", ["block", "point"])
def test_jacobi_csw0_is_neumann_series(kind):
    """c_SW = 0: A_D = 1 in both readings and M_j = sum_{i<j} (kappa H)^i."""
    op = _op(dims=(2, 4, 2, 2), kappa=0.11, csw=0.0, kind=kind)
    A = op.dense()
    KH = np.eye(op.N) - A                      # kappa H
    u = op.block_to_mat(wi.gaussian_block(op.V, 2, 10))
    want = sum(np.linalg.matrix_power(KH, i) @ u for i in range(6))
    got = jacobi_mat(op, u, 6)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13


def test_jacobi_converges_to_inverse_when_contracting():
    op = _op(dims=(2, 2, 4, 2), kappa=0.05, csw=1.0)
    A = op.dense()
    u = op.block_to_mat(wi.gaussian_block(op.V, 1, 11))
    x = np.linalg.solve(A, u)
    errs = [np.linalg.norm(jacobi_mat(op, u, j) - x) / np.linalg.norm(x) for j in (2, 6, 12)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


# ---------------------------------------------------------------- block BiCGGR

def _solve(op, B, j, **kw):
    return block_bicggr(op.A_mat, lambda m: jacobi_mat(op, m, j), B, kw.pop("tol", 1e-12), j, **kw)


@pytest.mark.parametrize("j,kind,L", [(0, "block", 3), (3, "block", 2), (2, "point", 3), (1, "block", 1)])
def test_bbicggr_matches_dense_lu_2x4(j, kind, L):
    op = _op(kappa=0.13, csw=1.5, kind=kind, eps=0.4)
    B = op.block_to_mat(wi.z4_block(op.V, L, 3))
    X, info = _solve(op, B, j)
    assert info["status"] == "converged"
    Xd = np.linalg.solve(op.dense(), B)
    assert np.max(true_residual(op.A_mat, B, X)) <= 1e-12
    cond = np.linalg.cond(op.dense())
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < cond * 1e-12


def test_bbicggr_small_workload_dense_lu():
    """4^4 lattice, kappa 0.12, c_SW 1.0, four Z4 sources, no preconditioner (N = 3072)."""
    w = wi.workload("lat4_L4_z4")
    op = WilsonClover(w["dims"], wi.random_links(w["dims"], w["eps"], w["link_seed"]), w["kappa"], w["csw"])
    B = op.block_to_mat(wi.z4_block(op.V, w["L"], w["source_seed"]))
    X, info = _solve(op, B, 0, tol=w["tol"])
    assert info["status"] == "converged"
    assert info["mvm_paper"] == 2 * info["iterations"] + 1
    assert np.max(true_residual(op.A_mat, B, X)) <= 1e-12
    Xd = np.linalg.solve(op.dense(), B)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 1e-10


@pytest.mark.parametrize("j", [0, 4])
def test_recursive_residual_tracks_true_residual(j):
    """R_k stays equal to B - A X_k up to rounding in every iteration."""
    op = _op(dims=(2, 2, 4, 4), kappa=0.125, csw=1.3)
    B = op.block_to_mat(wi.z4_block(op.V, 4, 12))
    bn = np.linalg.norm(B)
    gaps = []

    def cb(d):
        gaps.append(np.linalg.norm(d["Rn"] - (B - op.A_mat(d["X"]))) / bn)

    X, info = _solve(op, B, j, callback=cb)
    assert info["status"] == "converged"
    assert len(gaps) == info["iterations"]
    assert max(gaps) < 1e-13


def test_zeta_is_least_squares_minimiser():
    """zeta = Tr[W^H R]/Tr[W^H W] minimises ||R - zeta W||_F over complex zeta."""
    op = _op(dims=(2, 2, 2, 4), kappa=0.12, csw=1.0)
    B = op.block_to_mat(wi.gaussian_block(op.V, 3, 13))
    worst = []

    def cb(d):
        R, W, z = d["R"], d["W"], d["zeta"]
        f0 = np.linalg.norm(R - z * W)
        for dz in (1e-4, -1e-4, 1e-4j, -1e-4j):
            worst.append(np.linalg.norm(R - (z + dz * abs(z)) * W) - f0)

    _solve(op, B, 2, max_iter=6, callback=cb)
    assert min(worst) > 0


def test_alpha_solves_block_equation():
    op = _op(dims=(2, 2, 2, 4), kappa=0.12, csw=1.0)
    B = op.block_to_mat(wi.gaussian_block(op.V, 3, 14))
    errs = []

    def cb(d):
        errs.append(np.linalg.norm(d["C_v"] @ d["alpha"] - d["C_r"]) / np.linalg.norm(d["C_r"]))

    _solve(op, B, 1, max_iter=5, callback=cb)
    assert max(errs) < 1e-13


@pytest.mark.parametrize("j", [0, 1, 3])
def test_mvm_count_matches_table1_formula(j):
    """Counted operator applications per column equal 2(j+1)k + 1 at exit."""
    op = _op(dims=(2, 2, 2, 4), kappa=0.12, csw=1.0)
    B = op.block_to_mat(wi.z4_block(op.V, 2, 15))
    count = {"A": 0, "M": 0}

    def A(m):
        count["A"] += 1
        return op.A_mat(m)

    def M(m):
        count["M"] += 1
        return jacobi_mat(op, m, j)

    X, info = block_bicggr(A, M, B, 1e-12, j)
    assert info["status"] == "converged"
    k = info["iterations"]
    assert count["A"] + j * count["M"] == info["mvm_paper"] == 2 * (j + 1) * k + 1


def test_table1_entries_satisfy_mvm_formula():
    """Every printed (k, #MVM/L) pair of Table 1 obeys #MVM/L = 2(j+1)k + 1."""
    rows = np.loadtxt(os.path.join(HERE, "golden", "table1_iterations.txt"))
    assert rows.shape == (33, 4)
    for L, j, k, mvm in rows:
        assert abs(2 * (j + 1) * k + 1 - mvm) < 1e-6


def test_exact_preconditioner_converges_in_one_iteration():
    op = _op(kappa=0.13, csw=1.2)
    A = op.dense()
    Ainv = np.linalg.inv(A)
    B = op.block_to_mat(wi.z4_block(op.V, 3, 16))
    X, info = block_bicggr(op.A_mat, lambda m: Ainv @ m, B, 1e-12, 0)
    assert info["status"] == "converged" and info["iterations"] == 1
    assert np.linalg.norm(X - Ainv @ B) / np.linalg.norm(X) < 1e-13


def test_duplicate_columns_break_down():
    op = _op()
    b = wi.z4_block(op.V, 1, 17)
    B = op.block_to_mat(np.concatenate([b, b], axis=0))
    X, info = _solve(op, B, 1)
    assert info["status"] == "breakdown"
    assert np.all(np.isfinite(X))


def test_zero_column_rejected():
    op = _op()
    B = op.block_to_mat(wi.z4_block(op.V, 2, 18))
    B[:, 1] = 0
    with pytest.raises(ValueError):
        _solve(op, B, 0)


def test_max_iter_and_divergence_paths():
    op = _op(dims=(2, 2, 2, 4), kappa=0.12, csw=1.0)
    B = op.block_to_mat(wi.z4_block(op.V, 2, 19))
    X, info = _solve(op, B, 0, max_iter=3)
    assert info["status"] == "not_converged" and info["iterations"] == 3
    X, info = _solve(op, B, 0, diverge_at=1e-3)
    assert info["status"] == "diverged"


def test_restart_from_solution_is_immediate():
    op = _op()
    B = op.block_to_mat(wi.z4_block(op.V, 2, 20))
    Xd = np.linalg.solve(op.dense(), B)
    X, info = _solve(op, B, 2, X0=Xd)
    assert info["status"] == "converged" and info["iterations"] == 0
    X2, info2 = solve_with_restarts(op.A_mat, lambda m: jacobi_mat(op, m, 2), B, 1e-12, 2)
    assert info2["status"] == "converged"
    assert np.max(info2["true_residual"]) <= 1e-12


# ---------------------------------------------------------------- block BiCGSTAB (the foil)

from oracle.bicgstab import block_bicgstab  # noqa: E402


@pytest.mark.parametrize("j", [0, 2])
def test_bicgstab_single_column_matches_scipy(j):
    """L = 1: the block recurrences reduce to van der Vorst's BiCGSTAB; scipy's
    right-preconditioned implementation (r~ = r_0, x += alpha M p + omega M s) must produce the
    same iterates, which pins alpha, omega and the block form of beta."""
    import scipy.sparse.linalg as sla
    op = _op(dims=(2, 2, 4, 4), kappa=0.12, csw=1.1)
    N = op.N
    b = op.block_to_mat(wi.z4_block(op.V, 1, 41))
    Mf = (lambda m: jacobi_mat(op, m, j)) if j else (lambda m: m)
    Aop = sla.LinearOperator((N, N), matvec=lambda v: op.A_mat(v.reshape(N, 1))[:, 0], dtype=np.complex128)
    Mop = sla.LinearOperator((N, N), matvec=lambda v: Mf(v.reshape(N, 1))[:, 0], dtype=np.complex128)
    xs = []
    sla.bicgstab(Aop, b[:, 0], M=Mop, rtol=1e-30, atol=0.0, maxiter=8, callback=lambda x: xs.append(x.copy()))
    mine = []
    block_bicgstab(op.A_mat, Mf, b, 1e-30, j, max_iter=8, callback=lambda d: mine.append(d["X"][:, 0].copy()))
    assert len(xs) == 8 and len(mine) == 8
    for a, c in zip(mine, xs):
        assert np.linalg.norm(a - c) / np.linalg.norm(c) < 1e-11


@pytest.mark.parametrize("j,L", [(0, 3), (2, 2)])
def test_bicgstab_matches_dense_lu(j, L):
    op = _op(kappa=0.12, csw=1.2, eps=0.4)
    B = op.block_to_mat(wi.z4_block(op.V, L, 42))
    X, info = block_bicgstab(op.A_mat, lambda m: jacobi_mat(op, m, j), B, 1e-12, j)
    assert info["status"] == "converged"
    assert info["mvm_paper"] == 2 * (j + 1) * info["iterations"] + 1
    Xd = np.linalg.solve(op.dense(), B)
    cond = np.linalg.cond(op.dense())
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < cond * 1e-11


def test_bicgstab_exact_preconditioner_one_iteration():
    op = _op(kappa=0.13, csw=1.2)
    Ainv = np.linalg.inv(op.dense())
    B = op.block_to_mat(wi.z4_block(op.V, 3, 43))
    X, info = block_bicgstab(op.A_mat, lambda m: Ainv @ m, B, 1e-12, 0)
    assert info["status"] == "converged" and info["iterations"] == 1
    assert np.linalg.norm(X - Ainv @ B) / np.linalg.norm(X) < 1e-13
