"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the method (no Dirac operator, no
preconditioner, no solver step).  It only draws random numbers and lays
them out in the exchange formats defined by the C ABI:

* gauge links: complex128 array ``U[mu][site][a][b]`` of shape (4, V, 3, 3),
  ``U_mu(x)`` is the link from site x to x + mu-hat, mu = 0..3 = x, y, z, t;
* block vectors (N x L with N = 12 V): complex128 array of shape (L, 12, V),
  element ``[i, k, s]`` is column i, spin-colour component k = 3*spin + colour,
  site s;
* site index ``s = x + Lx*(y + Ly*(z + Lz*t))``.

The gauge ensemble stands in for the quenched configurations of the paper
(Sec. 3.1), which are not available: every link is ``exp(i eps H)`` with
``H`` a random traceless Hermitian 3x3 matrix ``sum_a h_a lambda_a / 2``,
``h_a`` i.i.d. standard normal (Gell-Mann matrices ``lambda_a``).
"""

from __future__ import annotations

import numpy as np

from .workloads import WORKLOADS, workload  # noqa: F401


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), normalised tr(l_a l_b) = 2 delta_ab."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _exp_i_eps_h(h: np.ndarray, eps: float, chunk: int = 1 << 20) -> np.ndarray:
    """exp(i*eps*H) for H = sum_a h[..., a] lambda_a / 2, batched over leading axes."""
    lam = gell_mann()
    flat = h.reshape(-1, 8)
    out = np.empty((flat.shape[0], 3, 3), dtype=np.complex128)
    for lo in range(0, flat.shape[0], chunk):
        hi = min(lo + chunk, flat.shape[0])
        H = np.einsum("na,aij->nij", flat[lo:hi], lam) * 0.5
        w, v = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        out[lo:hi] = np.einsum("nij,nj,nkj->nik", v, ph, v.conj())
    return out.reshape(h.shape[:-1] + (3, 3))


def random_links(dims, eps: float, seed: int) -> np.ndarray:
    """SU(3) links U = exp(i eps H), shape (4, V, 3, 3), complex128."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((4, V, 8))
    return _exp_i_eps_h(h, eps)


def random_gauge_transform(dims, eps: float, seed: int) -> np.ndarray:
    """One SU(3) matrix g(x) per site, shape (V, 3, 3), drawn like the links."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((V, 8))
    return _exp_i_eps_h(h, eps)


def gaussian_block(V: int, L: int, seed: int) -> np.ndarray:
    """Complex Gaussian block vector, shape (L, 12, V): re, im i.i.d. N(0, 1/2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((L, 12, V))
    im = rng.standard_normal((L, 12, V))
    return ((re + 1j * im) * np.sqrt(0.5)).astype(np.complex128)


def z4_block(V: int, L: int, seed: int) -> np.ndarray:
    """Z4-noise block vector, shape (L, 12, V): entries i.i.d. uniform on {1, i, -1, -i}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(0, 4, size=(L, 12, V))
    return (1j ** k).astype(np.complex128)


def point_block(V: int, L: int) -> np.ndarray:
    """Point sources, shape (L, 12, V): column i is the unit vector of spin-colour i at the origin.

    This is the source choice of the paper's tests (Sec. 3.3: b^(i) is the
    unit vector whose i-th component is one), with the first L of the twelve
    spin-colour components at site 0.
    """
    if L > 12:
        raise ValueError("point sources exist for L <= 12")
    b = np.zeros((L, 12, V), dtype=np.complex128)
    for i in range(L):
        b[i, i, 0] = 1.0
    return b


def source_block(kind: str, V: int, L: int, seed: int = 0) -> np.ndarray:
    if kind == "point":
        return point_block(V, L)
    if kind == "z4":
        return z4_block(V, L, seed)
    if kind == "gauss":
        return gaussian_block(V, L, seed)
    raise ValueError(f"unknown source kind {kind!r}")
