"""Linear gauge-covariant network used as a preconditioner, plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper leaves the search for a better preconditioner than Jacobi as
future work (Sec. 4) and requires only that M approximates A^{-1}
(Sec. 2).  The network used as such an M here is a product of three linear
layers; layer l maps a spinor field psi to

    (L_l psi)(x) = W_0 psi(x)
                   + sum_mu [ W_{+mu} U_mu(x) psi(x + mu)
                              + W_{-mu} U_mu(x - mu)^dag psi(x - mu) ]

with complex 4 x 4 matrices W acting on spin and the links acting on colour
(boundary conditions as for the operator).  M_theta = L_2 L_1 L_0.  The
parameters theta[l, d] are ordered d = 0 (site term), d = 1 + 2 mu (+mu),
d = 2 + 2 mu (-mu).  No bias and no nonlinearity: M_theta is linear, so the
block BiCGGR iteration stays valid with it as M.

Training minimises the mean over columns of ||M r - e||^2 / ||e||^2 for
pairs with A e = r (the error of the proposed correction), or of
||r - A M r||^2 / ||r||^2 (the residual the correction leaves, which is what a
preconditioner is for: it weights every eigenmode of A by its size in r
instead of by 1/lambda).  ``grad`` returns the real gradient packed as a complex
number, dl/d(Re W) + i dl/d(Im W) = 2 dl/d(conj W).  The adjoint layer is the
same layer with W_0 -> W_0^dag and W_{+-mu} -> W_{-+mu}^dag, because the
shift-with-link S_{+mu} has adjoint S_{-mu}.
"""

from __future__ import annotations

import numpy as np

from .dirac import dag, shift

NLAYER = 3
NDIR = 9


def identity_theta() -> np.ndarray:
    th = np.zeros((NLAYER, NDIR, 4, 4), dtype=np.complex128)
    th[:, 0] = np.eye(4)
    return th


def shifted(op, f: np.ndarray, d: int) -> np.ndarray:
    """S_d f: d = 0 identity, 1 + 2 mu: U_mu(x) f(x+mu), 2 + 2 mu: U_mu(x-mu)^dag f(x-mu)."""
    if d == 0:
        return f
    mu = (d - 1) // 2
    if d % 2 == 1:
        g = shift(f, mu, 1).copy()
        if mu == 3 and op.bc_t == 1:
            g[-1] *= -1.0
        return np.einsum("...ab,...sbl->...sal", op.U[mu], g)
    g = shift(f, mu, -1).copy()
    if mu == 3 and op.bc_t == 1:
        g[0] *= -1.0
    Ub = shift(op.U[mu], mu, -1)
    return np.einsum("...ba,...sbl->...sal", np.conj(Ub), g)


def layer(op, W: np.ndarray, f: np.ndarray) -> np.ndarray:
    """One layer with weights W (9, 4, 4) applied to an oracle field (..., 4, 3, L)."""
    out = np.zeros_like(f)
    for d in range(NDIR):
        out += np.einsum("st,...tal->...sal", W[d], shifted(op, f, d))
    return out


def layer_at(so, W: np.ndarray, s: int, get_spinor) -> np.ndarray:
    """One layer at a single site s, from the spinors of s and its eight
    neighbours: the same sum as ``layer`` with each term written as the
    Kronecker product (spin weight) x (link) acting on a (12, L) spinor
    (row 3*spin + colour).  ``so`` is a ``dirac.SiteOperator`` (links,
    coordinates, boundary signs); ``get_spinor(site)`` returns (12, L)."""
    c = so.coords(s)
    out = np.kron(W[0], np.eye(3)) @ get_spinor(s)
    for mu, d, sn, sign in so.neighbours(s):
        if d == 1:
            M = np.kron(W[1 + 2 * mu], so.link(mu, c))
        else:
            c_back = list(c)
            c_back[mu] -= 1
            M = np.kron(W[2 + 2 * mu], dag(so.link(mu, c_back)))
        out = out + sign * (M @ get_spinor(sn))
    return out


def adjoint_weights(W: np.ndarray) -> np.ndarray:
    Wa = np.empty_like(W)
    Wa[0] = W[0].conj().T
    for mu in range(4):
        Wa[1 + 2 * mu] = W[2 + 2 * mu].conj().T
        Wa[2 + 2 * mu] = W[1 + 2 * mu].conj().T
    return Wa


def forward(op, theta: np.ndarray, f: np.ndarray, keep: bool = False):
    zs = [f]
    for l in range(theta.shape[0]):
        zs.append(layer(op, theta[l], zs[-1]))
    return zs if keep else zs[-1]


def loss(op, theta, R: np.ndarray, E: np.ndarray) -> float:
    """Mean over columns of ||M r - e||^2 / ||e||^2 (R, E oracle fields with L columns)."""
    y = forward(op, theta, R)
    num = np.sum(np.abs(y - E) ** 2, axis=tuple(range(E.ndim - 1)))
    den = np.sum(np.abs(E) ** 2, axis=tuple(range(E.ndim - 1)))
    return float(np.mean(num / den))


def grad(op, theta, R: np.ndarray, E: np.ndarray):
    """(loss, gradient) with the gradient as dl/dRe + i dl/dIm, shape of theta."""
    zs = forward(op, theta, R, keep=True)
    y = zs[-1]
    axes = tuple(range(E.ndim - 1))
    den = np.sum(np.abs(E) ** 2, axis=axes)
    P = E.shape[-1]
    res = y - E
    lval = float(np.mean(np.sum(np.abs(res) ** 2, axis=axes) / den))
    g = res / den / P                       # dl/d(conj y)
    G = np.zeros_like(theta)
    for l in range(theta.shape[0] - 1, -1, -1):
        z = zs[l]
        for d in range(NDIR):
            sz = shifted(op, z, d)
            # dl/d(conj W_d) = sum_x,c,i g[s] conj(sz[s'])
            G[l, d] = 2.0 * np.einsum("nsal,ntal->st", g.reshape((-1,) + g.shape[-3:]),
                                      np.conj(sz).reshape((-1,) + sz.shape[-3:]))
        g = layer(op, adjoint_weights(theta[l]), g)
    return lval, G


def _gamma5(f: np.ndarray) -> np.ndarray:
    """gamma5 = diag(1, 1, -1, -1) on the spin index of an oracle field (chiral basis)."""
    out = f.copy()
    out[..., 2:, :, :] *= -1.0
    return out


def loss_residual(op, theta, R: np.ndarray) -> float:
    """Mean over columns of ||r - A M r||^2 / ||r||^2: the residual left after the correction M r
    that the preconditioner proposes for a residual r (for a pair with A e = r this is
    ||A (M r - e)||^2 / ||r||^2, the error measured in the residual norm)."""
    y = forward(op, theta, R)
    res = op.apply_A(y) - R
    axes = tuple(range(R.ndim - 1))
    return float(np.mean(np.sum(np.abs(res) ** 2, axis=axes) / np.sum(np.abs(R) ** 2, axis=axes)))


def grad_residual(op, theta, R: np.ndarray):
    """(loss_residual, gradient as dl/dRe + i dl/dIm).  dl/d(conj y) = A^H (A y - r) / ||r||^2 / P,
    with A^H = gamma5 A gamma5 (gamma5-hermiticity of the operator); then the same backward pass
    through the layers as ``grad``."""
    zs = forward(op, theta, R, keep=True)
    y = zs[-1]
    axes = tuple(range(R.ndim - 1))
    den = np.sum(np.abs(R) ** 2, axis=axes)
    P = R.shape[-1]
    res = op.apply_A(y) - R
    lval = float(np.mean(np.sum(np.abs(res) ** 2, axis=axes) / den))
    g = _gamma5(op.apply_A(_gamma5(res))) / den / P
    G = np.zeros_like(theta)
    for l in range(theta.shape[0] - 1, -1, -1):
        z = zs[l]
        for d in range(NDIR):
            sz = shifted(op, z, d)
            G[l, d] = 2.0 * np.einsum("nsal,ntal->st", g.reshape((-1,) + g.shape[-3:]),
                                      np.conj(sz).reshape((-1,) + sz.shape[-3:]))
        g = layer(op, adjoint_weights(theta[l]), g)
    return lval, G


def adam(theta, G, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the real and imaginary parts of theta (state: dict m, v, t)."""
    t = state.get("t", 0) + 1
    m = state.get("m", np.zeros_like(theta))
    v = state.get("v", np.zeros_like(theta))
    m = b1 * m + (1 - b1) * G
    v = b2 * v + (1 - b2) * (G.real ** 2 + 1j * G.imag ** 2)
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    step = mh.real / (np.sqrt(vh.real) + eps) + 1j * mh.imag / (np.sqrt(vh.imag) + eps)
    state.update(t=t, m=m, v=v)
    return theta - lr * step


def train(op, theta, R: np.ndarray, E: np.ndarray, steps: int, L: int, lr: float = 1e-3, residual: bool = False):
    """Adam for `steps` steps; batch b uses columns [b L, b L + L) (cycling).  residual: train on
    ``loss_residual`` (E unused) instead of ``loss``.  Returns (theta, losses)."""
    P = R.shape[-1]
    nb = max(1, P // L)
    state = {}
    hist = []
    for s in range(steps):
        b = s % nb
        sl = slice(b * L, b * L + L)
        lv, G = grad_residual(op, theta, R[..., sl]) if residual else grad(op, theta, R[..., sl], E[..., sl])
        hist.append(lv)
        theta = adam(theta, G, state, lr)
    return theta, hist
