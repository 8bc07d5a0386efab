"""Pins of the oracle's learned linear preconditioner: reduction to the Wilson
hopping term, identity initialisation, the adjoint identity, gauge
covariance, and central finite differences of the loss."""

import numpy as np
import pytest

import wdinputs as wi
from oracle import WilsonClover, gammas
from oracle import learned as ln


def _op(dims=(2, 2, 2, 4), kappa=0.11, csw=1.0, bc_t=1, seed=9):
    return WilsonClover(dims, wi.random_links(dims, 0.5, seed), kappa, csw, bc_t=bc_t)


def _rand_theta(rng, scale=0.3):
    th = ln.identity_theta()
    th += scale * (rng.standard_normal(th.shape) + 1j * rng.standard_normal(th.shape))
    return th


def test_identity_theta_is_identity():
    op = _op()
    f = op.from_block(wi.gaussian_block(op.V, 2, 1))
    assert np.array_equal(ln.forward(op, ln.identity_theta(), f), f)


@pytest.mark.parametrize("bc_t", [0, 1])
def test_layer_reduces_to_wilson_hop(bc_t):
    """W_0 = 1, W_{+mu} = kappa (1 - g_mu), W_{-mu} = kappa (1 + g_mu): the layer is 1 + kappa H."""
    op = _op(dims=(4, 2, 2, 4), kappa=0.13, csw=0.0, bc_t=bc_t)
    g = gammas()
    W = np.zeros((9, 4, 4), dtype=np.complex128)
    W[0] = np.eye(4)
    for mu in range(4):
        W[1 + 2 * mu] = op.kappa * (np.eye(4) - g[mu])
        W[2 + 2 * mu] = op.kappa * (np.eye(4) + g[mu])
    f = op.from_block(wi.gaussian_block(op.V, 3, 2))
    lhs = ln.layer(op, W, f)
    rhs = f + op.kappa * op.hop(f)
    assert np.max(np.abs(lhs - rhs)) < 1e-14
    # at c_SW = 0 this is 2 - A
    assert np.max(np.abs(lhs - (2 * f - op.apply_A(f)))) < 1e-14


def test_adjoint_identity():
    rng = np.random.default_rng(3)
    op = _op(dims=(2, 4, 2, 4))
    W = _rand_theta(rng)[0]
    phi = op.from_block(wi.gaussian_block(op.V, 2, 4))
    psi = op.from_block(wi.gaussian_block(op.V, 2, 5))
    lhs = np.vdot(phi, ln.layer(op, W, psi))
    rhs = np.vdot(ln.layer(op, ln.adjoint_weights(W), phi), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_gauge_covariance_and_linearity():
    rng = np.random.default_rng(6)
    dims = (2, 2, 4, 2)
    U = wi.random_links(dims, 0.5, 7)
    gx = wi.random_gauge_transform(dims, 1.0, 8)
    V = wi.volume(dims)
    lx, ly, lz, lt = dims
    Ug = np.empty_like(U)
    for s in range(V):
        c = [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]
        for mu in range(4):
            cn = list(c)
            cn[mu] = (cn[mu] + 1) % dims[mu]
            s2 = cn[0] + lx * (cn[1] + ly * (cn[2] + lz * cn[3]))
            Ug[mu, s] = gx[s] @ U[mu, s] @ gx[s2].conj().T
    op = WilsonClover(dims, U, 0.1, 1.0)
    opg = WilsonClover(dims, Ug, 0.1, 1.0)
    th = _rand_theta(rng)
    f = op.from_block(wi.gaussian_block(V, 2, 9))
    h = op.from_block(wi.gaussian_block(V, 2, 10))
    G = gx.reshape(op.shape + (3, 3))

    def gm(x):
        return np.einsum("...ab,...sbl->...sal", G, x)

    out = ln.forward(opg, th, gm(f))
    assert np.max(np.abs(out - gm(ln.forward(op, th, f)))) < 1e-13
    lin = ln.forward(op, th, 2.0 * f - 3j * h) - (2.0 * ln.forward(op, th, f) - 3j * ln.forward(op, th, h))
    assert np.max(np.abs(lin)) < 1e-12


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(11)
    op = _op(dims=(2, 2, 2, 2), bc_t=1)
    th = _rand_theta(rng, 0.2)
    R = op.from_block(wi.gaussian_block(op.V, 3, 12))
    E = op.from_block(wi.gaussian_block(op.V, 3, 13))
    lv, G = ln.grad(op, th, R, E)
    assert abs(lv - ln.loss(op, th, R, E)) < 1e-12
    h = 1e-6
    for _ in range(12):
        idx = tuple(rng.integers(0, n) for n in th.shape)
        for part in (1.0, 1j):
            tp = th.copy()
            tm = th.copy()
            tp[idx] += h * part
            tm[idx] -= h * part
            fd = (ln.loss(op, tp, R, E) - ln.loss(op, tm, R, E)) / (2 * h)
            an = G[idx].real if part == 1.0 else G[idx].imag
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_training_lowers_loss():
    op = _op(dims=(4, 4, 2, 2), kappa=0.1, csw=1.0, bc_t=0)
    E = op.from_block(wi.gaussian_block(op.V, 8, 14))
    R = op.apply_A(E)
    th0 = ln.identity_theta()
    l0 = ln.loss(op, th0, R, E)
    th, hist = ln.train(op, th0, R, E, steps=40, L=4, lr=1e-2)
    assert ln.loss(op, th, R, E) < 0.8 * l0


@pytest.mark.parametrize("bc_t", [0, 1])
def test_site_layer_matches_field_layer(bc_t):
    """The site-by-site layer (used for full-size spot checks) equals the field layer,
    on every site of a lattice with an odd extent and antiperiodic or periodic time."""
    from oracle.dirac import SiteOperator
    rng = np.random.default_rng(11)
    dims = (3, 2, 4, 4)
    U = wi.random_links(dims, 0.5, 21)
    op = WilsonClover(dims, U, 0.12, 1.0, bc_t=bc_t)
    so = SiteOperator(dims, U, 0.12, 1.0, bc_t)
    W = _rand_theta(rng)[1]
    b = wi.gaussian_block(op.V, 2, 8)                       # (L, 12, V)
    ref = op.to_block(ln.layer(op, W, op.from_block(b)))
    for s in range(op.V):
        got = ln.layer_at(so, W, s, lambda t: b[:, :, t].T)
        assert np.max(np.abs(got - ref[:, :, s].T)) < 1e-14


def test_adam_closed_form_steps():
    """Adam with bias correction, from its definition (not from the oracle's code): with a
    constant gradient the bias-corrected first and second moments equal g and g^2, so every
    step moves each real component by lr * g / (|g| + eps), i.e. lr * sign(g); with the
    gradient alternating g, -g the second step's corrected moments are
    m_hat = (0.9 * 0.1 - 0.1) g / (1 - 0.9^2) = -g / 19 and v_hat = g^2, a move of
    +lr / 19 * sign(g).  Real and imaginary parts are separate parameters."""
    lr = 1e-2
    g = np.array([[0.5 - 2.0j, -3.0 + 0.25j]])
    th0 = np.zeros_like(g)
    sign = np.sign(g.real) + 1j * np.sign(g.imag)
    # constant gradient: two steps of lr * sign(g) each (eps = 1e-8 is below 1e-7 relative here)
    st = {}
    th1 = ln.adam(th0, g, st, lr=lr)
    assert np.max(np.abs(th1 - (th0 - lr * sign))) < 1e-9
    th2 = ln.adam(th1, g, st, lr=lr)
    assert np.max(np.abs(th2 - (th0 - 2 * lr * sign))) < 1e-9
    # alternating gradient
    st = {}
    t1 = ln.adam(th0, g, st, lr=lr)
    t2 = ln.adam(t1, -g, st, lr=lr)
    assert np.max(np.abs((t2 - t1) - lr / 19.0 * sign)) < 1e-9
    assert st["t"] == 2


def test_residual_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(13)
    op = _op(dims=(2, 2, 2, 2), bc_t=1)
    th = _rand_theta(rng, 0.2)
    R = op.from_block(wi.gaussian_block(op.V, 3, 15))
    lv, G = ln.grad_residual(op, th, R)
    assert abs(lv - ln.loss_residual(op, th, R)) < 1e-12
    h = 1e-6
    for _ in range(12):
        idx = tuple(rng.integers(0, n) for n in th.shape)
        for part in (1.0, 1j):
            tp = th.copy()
            tm = th.copy()
            tp[idx] += h * part
            tm[idx] -= h * part
            fd = (ln.loss_residual(op, tp, R) - ln.loss_residual(op, tm, R)) / (2 * h)
            an = G[idx].real if part == 1.0 else G[idx].imag
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_residual_loss_closed_forms():
    """Closed forms: M = 1 leaves the residual r - A r; and for exact pairs (A e = r) the residual
    loss is the error of the correction measured through A, ||A (M r - e)||^2 / ||r||^2."""
    op = _op(dims=(2, 4, 2, 2), kappa=0.1, csw=0.0, bc_t=0)
    R = op.from_block(wi.gaussian_block(op.V, 2, 16))
    axes = tuple(range(R.ndim - 1))
    r2 = np.sum(np.abs(R) ** 2, axis=axes)
    want = np.mean(np.sum(np.abs(R - op.apply_A(R)) ** 2, axis=axes) / r2)
    assert abs(ln.loss_residual(op, ln.identity_theta(), R) - want) < 1e-14
    E = op.from_block(wi.gaussian_block(op.V, 2, 17))
    Rp = op.apply_A(E)
    th = _rand_theta(np.random.default_rng(2), 0.1)
    d = ln.forward(op, th, Rp) - E
    want = np.mean(np.sum(np.abs(op.apply_A(d)) ** 2, axis=axes) / np.sum(np.abs(Rp) ** 2, axis=axes))
    assert abs(ln.loss_residual(op, th, Rp) - want) < 1e-12 * max(1.0, want)
