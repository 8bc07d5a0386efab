"""Clover (O(a)-improved) Wilson-Dirac operator, plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper needs only that A is an N x N complex sparse non-Hermitian matrix
with N = Lx Ly Lz Lt * 3 * 4 (Sec. 2, eq. (1) and the dimension statement
after it) and leaves the explicit matrix to its companion paper.  The
convention fixed here is the textbook hopping-parameter form:

    (A psi)(x) = T(x) psi(x)
                 - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                    + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]

    T(x) = 1 - kappa c_SW sum_{mu < nu} sigma_{mu nu} (x) F_{mu nu}(x)
    sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu]
    F_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / (8 i)

with Q_{mu nu}(x) the sum of the four plaquettes in the mu-nu plane that
start and end at x, each traversed counter-clockwise (no trace subtraction).
Gamma matrices are the Euclidean chiral basis built from Pauli matrices:
gamma_k = [[0, -i s_k], [i s_k, 0]] (k = 1, 2, 3), gamma_4 = [[0, 1], [1, 0]].
The directions mu = 0, 1, 2, 3 are x, y, z, t and carry gamma_1..gamma_4.

Boundary conditions are periodic; with ``bc_t = 1`` the time direction is
antiperiodic: a hop across the t boundary picks up a factor -1.  The
clover term is unaffected since every closed loop crosses that boundary an
even number of times.

Fields are numpy arrays indexed [t, z, y, x, ...]; spinor fields carry
[..., spin(4), colour(3), column(L)].  Row n of the oracle's flattened N x L
matrices is 12*site + 3*spin + colour.
"""

from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# Spin algebra
# --------------------------------------------------------------------------

def pauli() -> np.ndarray:
    return np.array(
        [[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128
    )


def gammas() -> np.ndarray:
    """gamma_1..gamma_4 of the chiral basis, shape (4, 4, 4)."""
    s = pauli()
    z = np.zeros((2, 2), dtype=np.complex128)
    one = np.eye(2, dtype=np.complex128)
    g = [np.block([[z, -1j * s[k]], [1j * s[k], z]]) for k in range(3)]
    g.append(np.block([[z, one], [one, z]]))
    return np.array(g)


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def sigma_munu(mu: int, nu: int) -> np.ndarray:
    g = gammas()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


# --------------------------------------------------------------------------
# Geometry helpers
# --------------------------------------------------------------------------

def _axis(mu: int) -> int:
    # arrays are indexed [t, z, y, x]; direction mu = 0..3 is x, y, z, t
    return 3 - mu


def shift(f: np.ndarray, mu: int, step: int) -> np.ndarray:
    """g(x) = f(x + step * mu-hat) with periodic wrap-around."""
    return np.roll(f, -step, axis=_axis(mu))


def dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


# --------------------------------------------------------------------------
# The operator
# --------------------------------------------------------------------------

class WilsonClover:
    """A = T - kappa H on a periodic (optionally t-antiperiodic) 4-d lattice."""

    def __init__(self, dims, links_abi: np.ndarray, kappa: float, csw: float,
                 bc_t: int = 0, jacobi_kind: str = "block"):
        lx, ly, lz, lt = (int(d) for d in dims)
        self.dims = (lx, ly, lz, lt)
        self.shape = (lt, lz, ly, lx)
        self.V = lx * ly * lz * lt
        self.N = 12 * self.V
        self.kappa = float(kappa)
        self.csw = float(csw)
        self.bc_t = int(bc_t)
        self.jacobi_kind = jacobi_kind
        U = np.asarray(links_abi, dtype=np.complex128)
        assert U.shape == (4, self.V, 3, 3)
        self.U = U.reshape((4,) + self.shape + (3, 3))
        self.g = gammas()
        self.F = {}
        for mu in range(4):
            for nu in range(mu + 1, 4):
                self.F[(mu, nu)] = self.field_strength(mu, nu)
        self.T = self.site_matrix()
        self.Tinv = np.linalg.inv(self.T)
        self.Tdiag = np.real(np.einsum("...ii->...i", self.T)).copy()

    # ---- layout conversion (exchange format of the C ABI <-> oracle) ----
    def from_block(self, b: np.ndarray) -> np.ndarray:
        """(L, 12, V) exchange layout -> oracle field (Lt, Lz, Ly, Lx, 4, 3, L)."""
        L = b.shape[0]
        f = np.asarray(b).reshape((L, 4, 3) + self.shape)
        return np.ascontiguousarray(np.transpose(f, (3, 4, 5, 6, 1, 2, 0)))

    def to_block(self, f: np.ndarray) -> np.ndarray:
        """Oracle field -> (L, 12, V) exchange layout."""
        L = f.shape[-1]
        b = np.transpose(f, (6, 4, 5, 0, 1, 2, 3))
        return np.ascontiguousarray(b).reshape(L, 12, self.V)

    def to_matrix(self, f: np.ndarray) -> np.ndarray:
        return f.reshape(self.N, -1)

    def from_matrix(self, m: np.ndarray) -> np.ndarray:
        return m.reshape(self.shape + (4, 3, -1))

    # ---- clover ----
    def field_strength(self, mu: int, nu: int) -> np.ndarray:
        """F_{mu nu}(x) = (Q - Q^dag)/(8i), Q = sum of the four counter-clockwise leaves at x."""
        Umu, Unu = self.U[mu], self.U[nu]
        Umu_m = shift(Umu, mu, -1)             # U_mu(x - mu)
        Unu_m = shift(Unu, nu, -1)             # U_nu(x - nu)
        leaf1 = Umu @ shift(Unu, mu, 1) @ dag(shift(Umu, nu, 1)) @ dag(Unu)
        leaf2 = Unu @ dag(shift(Umu_m, nu, 1)) @ dag(shift(Unu, mu, -1)) @ Umu_m
        leaf3 = dag(Umu_m) @ dag(shift(shift(Unu, mu, -1), nu, -1)) @ shift(Umu_m, nu, -1) @ Unu_m
        leaf4 = dag(Unu_m) @ shift(Umu, nu, -1) @ shift(shift(Unu, mu, 1), nu, -1) @ dag(Umu)
        Q = leaf1 + leaf2 + leaf3 + leaf4
        return (Q - dag(Q)) / 8j

    def site_matrix(self) -> np.ndarray:
        """T(x) as a general 12 x 12 matrix per site, row/column index 3*spin + colour."""
        T = np.zeros(self.shape + (4, 3, 4, 3), dtype=np.complex128)
        for (mu, nu), F in self.F.items():
            s = sigma_munu(mu, nu)
            T -= self.kappa * self.csw * np.einsum("st,...ab->...satb", s, F)
        T = T.reshape(self.shape + (12, 12))
        T += np.eye(12)
        return T

    # ---- pieces of A ----
    def _site_mul(self, M: np.ndarray, f: np.ndarray) -> np.ndarray:
        L = f.shape[-1]
        v = f.reshape(self.shape + (12, L))
        return (M @ v).reshape(self.shape + (4, 3, L))

    def apply_T(self, f):
        return self._site_mul(self.T, f)

    def apply_Tinv(self, f):
        return self._site_mul(self.Tinv, f)

    def apply_Ddiag_inv(self, f):
        L = f.shape[-1]
        d = (1.0 / self.Tdiag).reshape(self.shape + (4, 3, 1))
        return f * d

    def apply_AD_inv(self, f):
        """A_D^{-1}: inverse of the diagonal part of A (site-block or point reading)."""
        if self.jacobi_kind == "block":
            return self.apply_Tinv(f)
        if self.jacobi_kind == "point":
            return self.apply_Ddiag_inv(f)
        raise ValueError(self.jacobi_kind)

    def hop(self, f: np.ndarray) -> np.ndarray:
        """H f = sum_mu [(1 - g_mu) U_mu(x) f(x+mu) + (1 + g_mu) U_mu(x-mu)^dag f(x-mu)]."""
        out = np.zeros_like(f)
        one = np.eye(4)
        for mu in range(4):
            fwd = shift(f, mu, 1).copy()
            bwd = shift(f, mu, -1).copy()
            if mu == 3 and self.bc_t == 1:
                fwd[-1] *= -1.0      # x + t-hat wraps from t = Lt-1 to t = 0
                bwd[0] *= -1.0       # x - t-hat wraps from t = 0 to t = Lt-1
            Ub = shift(self.U[mu], mu, -1)
            uf = np.einsum("...ab,...sbl->...sal", self.U[mu], fwd)
            ub = np.einsum("...ba,...sbl->...sal", np.conj(Ub), bwd)
            pm = one - self.g[mu]
            pp = one + self.g[mu]
            out += np.einsum("st,...tal->...sal", pm, uf)
            out += np.einsum("st,...tal->...sal", pp, ub)
        return out

    def apply_A(self, f: np.ndarray) -> np.ndarray:
        return self.apply_T(f) - self.kappa * self.hop(f)

    # ---- N x L matrix views used by the solver ----
    def A_mat(self, m: np.ndarray) -> np.ndarray:
        return self.to_matrix(self.apply_A(self.from_matrix(m)))

    def block_to_mat(self, b: np.ndarray) -> np.ndarray:
        return self.to_matrix(self.from_block(b))

    def mat_to_block(self, m: np.ndarray) -> np.ndarray:
        return self.to_block(self.from_matrix(m))

    # ---- dense assembly (small lattices only) ----
    def dense(self) -> np.ndarray:
        """A as a dense N x N matrix, column c = A e_c (oracle row order)."""
        if self.N > 4096:
            raise ValueError("dense assembly is for N <= 4096")
        eye = np.eye(self.N, dtype=np.complex128)
        return self.A_mat(eye)

    def point_index(self, site: int, spin: int, colour: int) -> int:
        return 12 * site + 3 * spin + colour


# --------------------------------------------------------------------------
# Single-site evaluation (for spot checks on lattices too large for the
# whole-lattice arrays above)
# --------------------------------------------------------------------------

class SiteOperator:
    """(A psi)(x) at individual sites, from the links around x only.

    Same definition as ``WilsonClover`` written site by site with explicit
    coordinates: the clover leaves at x are multiplied out link by link and
    the eight hops gather psi from the neighbours of x.  ``links_abi`` is the
    (4, V, 3, 3) exchange array; psi is read through ``get_spinor(site)``
    returning a (12, L) array (row 3*spin + colour).
    """

    def __init__(self, dims, links_abi, kappa, csw, bc_t=0):
        self.dims = tuple(int(d) for d in dims)
        self.U = links_abi
        self.kappa = float(kappa)
        self.csw = float(csw)
        self.bc_t = int(bc_t)
        self.g = gammas()

    def site(self, c):
        lx, ly, lz, lt = self.dims
        return (c[0] % lx) + lx * ((c[1] % ly) + ly * ((c[2] % lz) + lz * (c[3] % lt)))

    def coords(self, s):
        lx, ly, lz, lt = self.dims
        return [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]

    def link(self, mu, c):
        return self.U[mu, self.site(c)]

    @staticmethod
    def _mv(c, mu, d):
        c = list(c)
        c[mu] += d
        return c

    def field_strength(self, c, mu, nu):
        H = dag
        mv = self._mv
        lk = self.link
        l1 = lk(mu, c) @ lk(nu, mv(c, mu, 1)) @ H(lk(mu, mv(c, nu, 1))) @ H(lk(nu, c))
        l2 = lk(nu, c) @ H(lk(mu, mv(mv(c, mu, -1), nu, 1))) @ H(lk(nu, mv(c, mu, -1))) @ lk(mu, mv(c, mu, -1))
        l3 = H(lk(mu, mv(c, mu, -1))) @ H(lk(nu, mv(mv(c, mu, -1), nu, -1))) \
            @ lk(mu, mv(mv(c, mu, -1), nu, -1)) @ lk(nu, mv(c, nu, -1))
        l4 = H(lk(nu, mv(c, nu, -1))) @ lk(mu, mv(c, nu, -1)) @ lk(nu, mv(mv(c, mu, 1), nu, -1)) @ H(lk(mu, c))
        Q = l1 + l2 + l3 + l4
        return (Q - dag(Q)) / 8j

    def T(self, s):
        c = self.coords(s)
        T = np.eye(12, dtype=np.complex128)
        for mu in range(4):
            for nu in range(mu + 1, 4):
                T -= self.kappa * self.csw * np.kron(sigma_munu(mu, nu), self.field_strength(c, mu, nu))
        return T

    def neighbours(self, s):
        """[(mu, +1/-1, neighbour site, boundary sign)] for the eight hops of s."""
        c = self.coords(s)
        out = []
        lt = self.dims[3]
        for mu in range(4):
            for d in (1, -1):
                cn = self._mv(c, mu, d)
                sign = 1.0
                if self.bc_t and mu == 3 and (cn[3] == lt or cn[3] == -1):
                    sign = -1.0
                out.append((mu, d, self.site(cn), sign))
        return out

    def hop_at(self, s, get_spinor):
        """(H psi)(x) at site s, shape (12, L)."""
        c = self.coords(s)
        acc = None
        one = np.eye(4)
        for mu, d, sn, sign in self.neighbours(s):
            psi = get_spinor(sn)
            if d == 1:
                M = np.kron(one - self.g[mu], self.link(mu, c))
            else:
                M = np.kron(one + self.g[mu], dag(self.link(mu, self._mv(c, mu, -1))))
            term = sign * (M @ psi)
            acc = term if acc is None else acc + term
        return acc

    def apply_at(self, s, get_spinor):
        """(A psi)(x) at site s, shape (12, L)."""
        return self.T(s) @ get_spinor(s) - self.kappa * self.hop_at(s, get_spinor)
