"""Pins of the oracle's clover Wilson-Dirac operator against facts fixed
independently of its code: textbook gamma algebra, the free-field plane-wave
spectrum, gamma5-hermiticity, gauge covariance, a hand-derived single-link
clover field, and an element-by-element assembly written with explicit loops.
"""

import itertools

import numpy as np
import pytest

import wdinputs as wi
from oracle import WilsonClover, gammas, gamma5, sigma_munu

RTOL = 1e-13


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _unit_links(V):
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


# ---------------------------------------------------------------- gamma algebra

def test_gamma_clifford_and_hermitian():
    g = gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)


def test_gamma5_chiral_diagonal():
    # chiral basis: gamma5 = diag(1, 1, -1, -1)
    assert np.allclose(gamma5(), np.diag([1, 1, -1, -1]), atol=1e-15)


def test_sigma_block_structure():
    # sigma_{mu nu} commutes with gamma5, so it is block diagonal in the chiral basis
    g5 = gamma5()
    for mu, nu in itertools.combinations(range(4), 2):
        s = sigma_munu(mu, nu)
        assert np.allclose(s @ g5, g5 @ s, atol=1e-15)
        assert np.allclose(s, s.conj().T, atol=1e-15)


# ---------------------------------------------------------------- free field

@pytest.mark.parametrize("dims,bc_t", [((4, 4, 4, 4), 0), ((3, 4, 5, 6), 1), ((2, 2, 2, 2), 0)])
def test_free_field_plane_wave(dims, bc_t):
    """Unit links: A e^{ipx} u = [1 - 2k sum cos p + 2ik sum gamma_mu sin p_mu] e^{ipx} u."""
    kappa = 0.137
    V = wi.volume(dims)
    op = WilsonClover(dims, _unit_links(V), kappa, csw=1.7, bc_t=bc_t)
    rng = np.random.default_rng(3)
    g = gammas()
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    for _ in range(4):
        n = [rng.integers(0, d) for d in dims]
        p = [2 * np.pi * n[m] / dims[m] for m in range(4)]
        if bc_t:
            p[3] = np.pi * (2 * n[3] + 1) / lt
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        psi = phase[..., None, None, None] * u[None, None, None, None, :, :, None]
        out = op.apply_A(psi)
        M = (1 - 2 * kappa * sum(np.cos(pm) for pm in p)) * np.eye(4) + \
            2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = phase[..., None, None, None] * (M @ u)[None, None, None, None, :, :, None]
        assert _rel(out, expect) < RTOL


def test_free_field_spectrum_dense():
    """Eigenvalues of the free operator: 1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p), six-fold each."""
    dims, kappa = (3, 3, 3, 4), 0.11
    V = wi.volume(dims)
    op = WilsonClover(dims, _unit_links(V), kappa, csw=1.0, bc_t=1)
    ev = np.linalg.eigvals(op.dense())
    expect = []
    for n in itertools.product(*(range(d) for d in dims)):
        p = [2 * np.pi * n[m] / dims[m] for m in range(3)] + [np.pi * (2 * n[3] + 1) / dims[3]]
        re = 1 - 2 * kappa * sum(np.cos(q) for q in p)
        im = 2 * kappa * np.sqrt(sum(np.sin(q) ** 2 for q in p))
        expect += [re + 1j * im] * 6 + [re - 1j * im] * 6
    expect = np.array(expect)

    def canon(z):
        return z[np.lexsort((np.round(z.imag, 8), np.round(z.real, 8)))]

    assert np.max(np.abs(canon(ev) - canon(expect))) < 1e-10


# ---------------------------------------------------------------- symmetries

@pytest.mark.parametrize("bc_t", [0, 1])
def test_gamma5_hermiticity(bc_t):
    dims = (4, 4, 2, 6)
    U = wi.random_links(dims, 0.4, 11)
    op = WilsonClover(dims, U, 0.13, 1.6, bc_t=bc_t)
    g5 = gamma5()
    phi = op.from_block(wi.gaussian_block(op.V, 2, 12))
    psi = op.from_block(wi.gaussian_block(op.V, 2, 13))

    def g5a(f):
        return np.einsum("st,...tal->...sal", g5, f)

    lhs = np.vdot(phi, g5a(op.apply_A(g5a(psi))))
    rhs = np.vdot(op.apply_A(phi), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14


@pytest.mark.parametrize("bc_t", [0, 1])
def test_gauge_covariance(bc_t):
    """A[U^g](g psi) = g A[U] psi for U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    dims = (4, 2, 4, 4)
    V = wi.volume(dims)
    U = wi.random_links(dims, 0.5, 21)
    gx = wi.random_gauge_transform(dims, 1.0, 22)
    lx, ly, lz, lt = dims
    Ug = np.empty_like(U)
    for s in range(V):
        x, y, z, t = s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)
        for mu in range(4):
            c = [x, y, z, t]
            c[mu] = (c[mu] + 1) % dims[mu]
            s2 = c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))
            Ug[mu, s] = gx[s] @ U[mu, s] @ gx[s2].conj().T
    op = WilsonClover(dims, U, 0.125, 1.3, bc_t=bc_t)
    opg = WilsonClover(dims, Ug, 0.125, 1.3, bc_t=bc_t)
    psi = op.from_block(wi.gaussian_block(V, 3, 23))
    G = gx.reshape(op.shape + (3, 3))

    def gmul(f):
        return np.einsum("...ab,...sbl->...sal", G, f)

    assert _rel(opg.apply_A(gmul(psi)), gmul(op.apply_A(psi))) < RTOL


# ---------------------------------------------------------------- clover isolation

def test_kappa_zero_is_identity_and_csw_zero_is_wilson():
    dims = (2, 4, 2, 4)
    U = wi.random_links(dims, 0.5, 31)
    psi_b = wi.gaussian_block(wi.volume(dims), 2, 32)
    op0 = WilsonClover(dims, U, 0.0, 1.5)
    f = op0.from_block(psi_b)
    assert np.array_equal(op0.apply_A(f), f)
    opw = WilsonClover(dims, U, 0.12, 0.0)
    assert np.allclose(opw.T, np.eye(12), atol=0)


def test_site_matrix_hermitian_chiral_blocks():
    dims = (4, 4, 4, 4)
    op = WilsonClover(dims, wi.random_links(dims, 0.3, 41), 0.12, 1.0)
    T = op.T
    assert np.max(np.abs(T - np.conj(np.swapaxes(T, -1, -2)))) == 0.0
    blk = T.reshape(op.shape + (2, 6, 2, 6))
    assert np.max(np.abs(blk[..., 0, :, 1, :])) == 0.0
    assert np.max(np.abs(blk[..., 1, :, 0, :])) == 0.0


def test_single_link_clover_closed_form():
    """All links 1 except U_x(x0) = diag(e^{i phi}, e^{-i phi}, 1).

    Hand derivation: the only plaquettes that differ from 1 are the two in
    each (x, nu) plane that contain the modified link.  The clover sum at
    x0 + nu-hat contains one leaf equal to D = U_x(x0), so
    F_{x nu}(x0 + nu) = (D - D^dag)/(8i) = (sin(phi)/4) diag(1, -1, 0); at
    x0 - nu the leaf is D^dag and the sign flips; at x0 and x0 + x-hat both
    leaves appear and cancel.  With sigma_{x nu} for nu = y, z, t equal to
    -diag(s3, s3), diag(s2, s2) and diag(s1, -s1) in the chiral basis,
    T = 1 - kappa c_SW sigma_{x nu} F_{x nu} at those sites.
    """
    dims = (4, 4, 4, 4)
    V = wi.volume(dims)
    phi, kappa, csw = 0.7, 0.13, 1.9
    x0 = (1, 2, 1, 3)

    def site(c):
        c = [c[m] % dims[m] for m in range(4)]
        return c[0] + 4 * (c[1] + 4 * (c[2] + 4 * c[3]))

    U = _unit_links(V)
    D = np.diag([np.exp(1j * phi), np.exp(-1j * phi), 1.0])
    U[0, site(x0)] = D
    op = WilsonClover(dims, U, kappa, csw)
    Tflat = op.T.reshape(V, 12, 12)
    f = np.sin(phi) / 4 * np.diag([1.0, -1.0, 0.0])
    s1 = np.array([[0, 1], [1, 0]])
    s2 = np.array([[0, -1j], [1j, 0]])
    s3 = np.array([[1, 0], [0, -1]])
    z2 = np.zeros((2, 2))
    sig = {1: -np.block([[s3, z2], [z2, s3]]),
           2: np.block([[s2, z2], [z2, s2]]),
           3: np.block([[s1, z2], [z2, -s1]])}
    expected = {s: np.eye(12, dtype=complex) for s in range(V)}
    for nu in (1, 2, 3):
        for sign in (+1, -1):
            c = list(x0)
            c[nu] += sign
            expected[site(c)] = expected[site(c)] - kappa * csw * sign * np.kron(sig[nu], f)
            c2 = list(c)
            c2[0] += 1
            expected[site(c2)] = expected[site(c2)] - kappa * csw * sign * np.kron(sig[nu], f)
    err = max(np.max(np.abs(Tflat[s] - expected[s])) for s in range(V))
    assert err < 1e-15
    # x0 and x0 + x-hat see both leaves: no field there
    assert np.allclose(Tflat[site(x0)], np.eye(12), atol=1e-16)
    assert np.allclose(Tflat[site((x0[0] + 1,) + x0[1:])], np.eye(12), atol=1e-16)


# ---------------------------------------------------------------- explicit-loop assembly

def _brute_dense(dims, U, kappa, csw, bc_t):
    """A assembled element by element with coordinate arithmetic (no array shifts)."""
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    s1 = np.array([[0, 1], [1, 0]], dtype=complex)
    s2 = np.array([[0, -1j], [1j, 0]])
    s3 = np.array([[1, 0], [0, -1]], dtype=complex)
    z2 = np.zeros((2, 2))
    e2 = np.eye(2)
    gam = [np.block([[z2, -1j * s], [1j * s, z2]]) for s in (s1, s2, s3)]
    gam.append(np.block([[z2, e2], [e2, z2]]))

    def coords(s):
        return [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]

    def site(c):
        return (c[0] % lx) + lx * ((c[1] % ly) + ly * ((c[2] % lz) + lz * (c[3] % lt)))

    def link(mu, c):
        return U[mu, site(c)]

    def mv(c, mu, d):
        c = list(c)
        c[mu] += d
        return c

    N = 12 * V
    A = np.zeros((N, N), dtype=complex)
    for s in range(V):
        c = coords(s)
        T = np.eye(12, dtype=complex)
        for mu in range(4):
            for nu in range(mu + 1, 4):
                H = lambda M: M.conj().T  # noqa: E731
                l1 = link(mu, c) @ link(nu, mv(c, mu, 1)) @ H(link(mu, mv(c, nu, 1))) @ H(link(nu, c))
                l2 = link(nu, c) @ H(link(mu, mv(mv(c, mu, -1), nu, 1))) @ H(link(nu, mv(c, mu, -1))) \
                    @ link(mu, mv(c, mu, -1))
                l3 = H(link(mu, mv(c, mu, -1))) @ H(link(nu, mv(mv(c, mu, -1), nu, -1))) \
                    @ link(mu, mv(mv(c, mu, -1), nu, -1)) @ link(nu, mv(c, nu, -1))
                l4 = H(link(nu, mv(c, nu, -1))) @ link(mu, mv(c, nu, -1)) \
                    @ link(nu, mv(mv(c, mu, 1), nu, -1)) @ H(link(mu, c))
                Q = l1 + l2 + l3 + l4
                F = (Q - Q.conj().T) / 8j
                sg = 0.5j * (gam[mu] @ gam[nu] - gam[nu] @ gam[mu])
                T -= kappa * csw * np.kron(sg, F)
        A[12 * s:12 * s + 12, 12 * s:12 * s + 12] += T
        for mu in range(4):
            cf = mv(c, mu, 1)
            cb = mv(c, mu, -1)
            sf = -1.0 if (bc_t and mu == 3 and cf[3] == lt) else 1.0
            sb = -1.0 if (bc_t and mu == 3 and cb[3] == -1) else 1.0
            f, b = site(cf), site(cb)
            A[12 * s:12 * s + 12, 12 * f:12 * f + 12] += -kappa * sf * np.kron(np.eye(4) - gam[mu], link(mu, c))
            A[12 * s:12 * s + 12, 12 * b:12 * b + 12] += -kappa * sb * np.kron(np.eye(4) + gam[mu],
                                                                             link(mu, cb).conj().T)
    return A


@pytest.mark.parametrize("dims,bc_t", [((2, 2, 2, 2), 0), ((2, 3, 2, 3), 1)])
def test_dense_matches_explicit_loops(dims, bc_t):
    U = wi.random_links(dims, 0.6, 51)
    op = WilsonClover(dims, U, 0.14, 1.4, bc_t=bc_t)
    assert np.max(np.abs(op.dense() - _brute_dense(dims, U, 0.14, 1.4, bc_t))) < 1e-14


def test_diagonal_blocks_of_dense_are_T():
    """A_D (site-block reading) is exactly the 12 x 12 diagonal block of A, also on extent-2 lattices."""
    dims = (2, 2, 2, 2)
    op = WilsonClover(dims, wi.random_links(dims, 0.6, 61), 0.14, 1.4)
    D = op.dense()
    Tflat = op.T.reshape(op.V, 12, 12)
    for s in range(op.V):
        assert np.max(np.abs(D[12 * s:12 * s + 12, 12 * s:12 * s + 12] - Tflat[s])) < 1e-15


def test_layout_roundtrip_and_point_source():
    dims = (2, 3, 4, 5)
    op = WilsonClover(dims, _unit_links(wi.volume(dims)), 0.1, 1.0)
    b = wi.gaussian_block(op.V, 3, 71)
    assert np.array_equal(op.to_block(op.from_block(b)), b)
    # exchange-format element [i, k, s] is oracle row 12 s + k of column i
    m = op.block_to_mat(b)
    assert m[12 * 7 + 5, 2] == b[2, 5, 7]
    pb = wi.point_block(op.V, 12)
    pm = op.block_to_mat(pb)
    assert np.array_equal(pm, np.eye(op.N, 12))


# ------------------------------------------------- site-by-site operator

@pytest.mark.parametrize("dims,bc_t", [((3, 5, 3, 5), 0), ((3, 5, 3, 5), 1), ((2, 2, 2, 2), 0),
                                       ((2, 2, 2, 2), 1)])
def test_site_operator_matches_field_operator(dims, bc_t):
    """SiteOperator (used for the full-size spot checks on the GPU) builds T from its own
    link-by-link leaves and the hop from kron((1 -+ g_mu), U) products; at every site of an
    odd-extent lattice and of 2^4 (where x + mu = x - mu and both hops add) its T, hop and
    A psi equal the field operator's, which the closed forms above pin."""
    from oracle.dirac import SiteOperator
    U = wi.random_links(dims, 0.4, 31 + bc_t)
    kappa, csw = 0.124, 1.3
    op = WilsonClover(dims, U, kappa, csw, bc_t=bc_t)
    so = SiteOperator(dims, U, kappa, csw, bc_t)
    b = wi.gaussian_block(op.V, 3, 17)
    f = op.from_block(b)
    H = op.to_block(op.hop(f))
    A = op.to_block(op.apply_A(f))
    T = op.T.reshape(op.V, 12, 12)   # oracle field order is [t, z, y, x] = site order
    get = lambda s: b[:, :, s].T      # (12, L) at site s
    for s in range(op.V):
        assert np.max(np.abs(so.T(s) - T[s])) < 1e-15
        assert _rel(so.hop_at(s, get), H[:, :, s].T) < 1e-14
        assert _rel(so.apply_at(s, get), A[:, :, s].T) < 1e-14
