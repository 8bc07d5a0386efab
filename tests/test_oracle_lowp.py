"""Pins of the oracle's low-precision operator and Jacobi sweeps (the reference of
the mixed-precision extension): bfloat16 round-to-nearest-even on hand-picked
values, the "f64" format reproducing the FP64 operator and the paper's closed-form
Jacobi sum, and the FP32 / BF16 formats staying within the rounding bounds derived
from the storage formats (u = 2^-24 and 2^-8)."""

import numpy as np
import pytest

import wdinputs as wi
from oracle import WilsonClover
from oracle.jacobi import jacobi_apply
from oracle.lowp import apply_lowp, jacobi_sweeps_lowp, round_bf16, store

U32, UBF = 2.0 ** -24, 2.0 ** -8


def test_bf16_round_to_nearest_even():
    x = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, 1 + 2 ** -7 + 2 ** -20, -2.5, 3 * 2 ** -130],
                 dtype=np.float32)
    want = np.array([1.0, 1 + 2 ** -6, 1.0, 1 + 2 ** -7, -2.5, 3 * 2 ** -130], dtype=np.float32)
    assert np.array_equal(round_bf16(x), want)
    r = round_bf16(np.random.default_rng(1).standard_normal(1000).astype(np.float32))
    assert np.all(r.view(np.uint32) & 0xFFFF == 0)
    assert np.array_equal(round_bf16(r), r)


def _op(bc_t=1):
    dims = (4, 4, 2, 6)
    return WilsonClover(dims, wi.random_links(dims, 0.3, 311), 0.127, 1.6, bc_t=bc_t)


@pytest.mark.parametrize("bc_t", [0, 1])
def test_f64_format_is_the_fp64_operator_and_closed_form(bc_t):
    op = _op(bc_t)
    X = op.from_block(wi.gaussian_block(op.V, 3, 312))
    A = op.apply_A(X)
    assert np.max(np.abs(apply_lowp(op, X, "f64") - A)) < 1e-13 * np.max(np.abs(A))
    for j in (1, 2, 5):
        ref = jacobi_apply(op, X, j)        # the paper's sum, term by term
        got = jacobi_sweeps_lowp(op, X, j, "f64")
        assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("fmt,u", [("f32", U32), ("bf16", UBF)])
def test_low_formats_within_rounding_bounds(fmt, u):
    """Every stored factor carries a relative rounding of at most u and each product two of
    them; with sum|terms| / |result| ~ 3 the max error relative to the largest output stays
    below 9 u per application (BF16; float32 accumulation adds ~100 u32 for FP32), and the
    stored iterates add one rounding per sweep.  The errors must also not vanish, which
    would mean the format was not applied."""
    op = _op()
    X = op.from_block(wi.gaussian_block(op.V, 3, 313))
    A = op.apply_A(X)
    bound = 9 * u if fmt == "bf16" else 1e3 * u
    e = np.max(np.abs(apply_lowp(op, X, fmt) - A)) / np.max(np.abs(A))
    assert u / 100 < e < bound
    for j in (1, 3):
        ref = jacobi_apply(op, X, j)
        e = np.max(np.abs(jacobi_sweeps_lowp(op, X, j, fmt) - ref)) / np.max(np.abs(ref))
        assert u / 100 < e < j * bound
    s = store(X, fmt)
    assert s.dtype == np.complex64 and np.array_equal(store(s, fmt), s)


def test_third_row_of_links_is_conjugate_cross_product():
    """The synthetic links exp(i eps H), H traceless Hermitian, lie in SU(3): unitary with unit
    determinant, so row 2 = conj(row 0 x row 1) -- the identity the two-row link storage of the
    FP32 / BF16 formats relies on."""
    U = wi.random_links((4, 4, 2, 4), 0.4, 315)
    r2 = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    assert np.max(np.abs(r2 - U[..., 2, :])) < 1e-13
    assert np.max(np.abs(np.linalg.det(U) - 1.0)) < 1e-13
