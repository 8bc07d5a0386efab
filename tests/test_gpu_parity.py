"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: FP64 operator and preconditioner applications agree with the
oracle to 1e-13 relative (each output element is a short fixed sum, so the
only difference is rounding order, ~1e-16 per element); solves reach a true
residual <= 1e-12 per column, checked with the oracle's own operator.
"""

import sys

import numpy as np
import pytest

import wdinputs as wi
from oracle import WilsonClover, gamma5
from oracle.dirac import SiteOperator
from oracle.jacobi import jacobi_apply
from oracle.bbicggr import block_bicggr, true_residual

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    sys.__stderr__.write(f"[gpu] {msg}\n")
    sys.__stderr__.flush()


@pytest.fixture(autouse=True)
def _announce(request):
    _say(request.node.nodeid)
    yield


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0907_3261_amd as p
    p.load()
    return p


def _ctx(pkg, dims, U, kappa, csw, bc_t=0, max_L=12, kind=0):
    c = pkg.Context(dims, bc_t=bc_t, max_L=max_L)
    c.set_links(U)
    c.set_params(kappa, csw, kind)
    return c


def _dev(b):
    return torch.from_numpy(np.ascontiguousarray(b)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _maxrel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


# Site maps exercised: (2, 2, 2, 2) the plain linear order (too small to split over the 8 XCDs);
# (8, 16, 8, 3) the y x z = 1 x 8 split; (4, 4, 4, 4), (8, 6, 4, 10) and (16, 8, 4, 4) the 2 x 4
# split with one z plane per XCD; (3, 4, 5, 6) the 2 x 4 split with uneven y and z ranges.
CASES = [((4, 4, 4, 4), 0), ((3, 4, 5, 6), 1), ((2, 2, 2, 2), 0), ((8, 6, 4, 10), 1), ((16, 8, 4, 4), 1),
         ((8, 16, 8, 3), 0)]


# ---------------------------------------------------------------- clover setup

@pytest.mark.parametrize("dims,bc_t", CASES)
def test_clover_and_inverse(pkg, dims, bc_t):
    U = wi.random_links(dims, 0.4, 101)
    op = WilsonClover(dims, U, 0.13, 1.6, bc_t=bc_t)
    c = _ctx(pkg, dims, U, 0.13, 1.6, bc_t)
    T = c.clover(0)
    Ti = c.clover(1)
    Tor = op.T.reshape(op.V, 12, 12)
    Tior = op.Tinv.reshape(op.V, 12, 12)
    for ch in range(2):
        sl = slice(6 * ch, 6 * ch + 6)
        assert np.max(np.abs(T[:, ch] - Tor[:, sl, sl])) < 1e-14
        assert _maxrel(Ti[:, ch], Tior[:, sl, sl]) < 1e-13
    c.close()


# ---------------------------------------------------------------- operator

@pytest.mark.parametrize("dims,bc_t", CASES)
@pytest.mark.parametrize("L", [1, 4, 5, 12])
def test_apply_matches_oracle(pkg, dims, bc_t, L):
    U = wi.random_links(dims, 0.4, 102)
    op = WilsonClover(dims, U, 0.128, 1.6, bc_t=bc_t)
    c = _ctx(pkg, dims, U, 0.128, 1.6, bc_t, max_L=12)
    X = wi.gaussian_block(op.V, L, 103)
    Y = _host(c.apply(_dev(X)))
    Yo = op.to_block(op.apply_A(op.from_block(X)))
    assert _maxrel(Y, Yo) < 1e-13
    for i in range(L):
        assert _rel(Y[i], Yo[i]) < 1e-13
    c.close()


def test_apply_max_columns_and_ragged_volume(pkg):
    dims = (5, 3, 3, 5)           # V = 225: not a multiple of the 64-site tile
    U = wi.random_links(dims, 0.4, 104)
    op = WilsonClover(dims, U, 0.12, 1.0)
    c = _ctx(pkg, dims, U, 0.12, 1.0, max_L=16)
    X = wi.gaussian_block(op.V, 16, 105)
    Y = _host(c.apply(_dev(X)))
    assert _maxrel(Y, op.to_block(op.apply_A(op.from_block(X)))) < 1e-13
    c.close()


def test_apply_gamma5_hermiticity_and_determinism(pkg):
    dims = (4, 4, 4, 8)
    U = wi.random_links(dims, 0.3, 106)
    c = _ctx(pkg, dims, U, 0.135, 1.6, 1)
    V = wi.volume(dims)
    phi = wi.gaussian_block(V, 3, 107)
    psi = wi.gaussian_block(V, 3, 108)
    g5 = np.diag(gamma5()).real                       # +1, +1, -1, -1
    g5k = np.repeat(g5, 3)[None, :, None]             # per component k = 3*spin + colour
    Ag5psi = _host(c.apply(_dev(g5k * psi)))
    Aphi = _host(c.apply(_dev(phi)))
    lhs = np.vdot(phi, g5k * Ag5psi)
    rhs = np.vdot(Aphi, psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    Aphi2 = _host(c.apply(_dev(phi)))
    assert np.array_equal(Aphi, Aphi2)
    c.close()


def test_apply_rejects_bad_arguments(pkg):
    dims = (4, 4, 4, 4)
    c = pkg.Context(dims, max_L=4)
    X = c.empty_block(2)
    with pytest.raises(pkg.WDError):          # parameters not set yet
        c.apply(X)
    c.set_links(wi.random_links(dims, 0.3, 1))
    c.set_params(0.12, 1.0)
    with pytest.raises(pkg.WDError):          # L above max_L
        c.apply(c.empty_block(5))
    with pytest.raises(pkg.WDError):          # output aliases input
        c.apply(X, X)
    c.close()


# ---------------------------------------------------------------- Jacobi

@pytest.mark.parametrize("L", [2, 3, 7])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("j", [0, 1, 2, 5, 12])
@pytest.mark.parametrize("dims", [(4, 4, 6, 4), (8, 16, 8, 3)])
def test_jacobi_matches_oracle(pkg, kind, j, dims, L):
    """Both A_D readings; L = 2 runs the register-tiled sweep, L = 3 and 7 the LDS-staged one (whose
    four waves then take one, or two and one, columns each)."""
    U = wi.random_links(dims, 0.3, 109)
    op = WilsonClover(dims, U, 0.13, 1.6, bc_t=1, jacobi_kind="block" if kind == 0 else "point")
    c = _ctx(pkg, dims, U, 0.13, 1.6, 1, kind=kind)
    R = wi.gaussian_block(op.V, L, 110)
    Z = _host(c.jacobi(_dev(R), j))
    Zo = op.to_block(jacobi_apply(op, op.from_block(R), j))
    assert _maxrel(Z, Zo) < 1e-13
    c.close()


# ---------------------------------------------------------------- block kernels

@pytest.mark.parametrize("L", [1, 3, 12, 16])
def test_block_gram(pkg, L):
    dims = (3, 5, 4, 7)
    c = pkg.Context(dims, max_L=16)
    V = wi.volume(dims)
    P = wi.gaussian_block(V, L, 111)
    Q = wi.gaussian_block(V, L, 112)
    C = _host(c.gram(_dev(P), _dev(Q)))
    Pm = P.reshape(L, -1).T
    Qm = Q.reshape(L, -1).T
    Co = Pm.conj().T @ Qm
    assert _maxrel(C, Co) < 1e-13
    c.close()


def test_block_gram_large_rows(pkg):
    dims = (16, 16, 16, 8)        # N = 393216 rows: many partial blocks
    c = pkg.Context(dims, max_L=12)
    V = wi.volume(dims)
    P = wi.gaussian_block(V, 12, 113)
    Q = wi.gaussian_block(V, 12, 114)
    C = _host(c.gram(_dev(P), _dev(Q)))
    Co = P.reshape(12, -1).conj() @ Q.reshape(12, -1).T
    assert _maxrel(C, Co) < 1e-13
    c.close()


@pytest.mark.parametrize("L", [1, 2, 7, 12, 16])
def test_small_solve(pkg, L):
    c = pkg.Context((2, 2, 2, 2), max_L=16)
    rng = np.random.default_rng(L)
    M = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))
    B = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))
    Z, ok = c.small_solve(_dev(M), _dev(B))
    assert ok
    assert _maxrel(_host(Z), np.linalg.solve(M, B)) < 1e-11
    if L > 1:
        Ms = M.copy()
        Ms[1] = Ms[0]             # exactly singular
        Z, ok = c.small_solve(_dev(Ms), _dev(B))
        assert not ok
    c.close()


# ---------------------------------------------------------------- solver

def _workload_ctx(pkg, name):
    w = wi.workload(name)
    U = wi.random_links(w["dims"], w["eps"], w["link_seed"])
    kappa = w["kappa"] if not isinstance(w["kappa"], tuple) else w["kappa"][0]
    c = _ctx(pkg, w["dims"], U, kappa, w["csw"], w["bc_t"], max_L=12)
    op = WilsonClover(w["dims"], U, kappa, w["csw"], bc_t=w["bc_t"])
    return w, c, op


def test_solve_small_workload_matches_dense_lu(pkg):
    """4^4, kappa 0.12, c_SW 1.0, four Z4 sources, no preconditioner."""
    w, c, op = _workload_ctx(pkg, "lat4_L4_z4")
    B = wi.z4_block(op.V, w["L"], w["source_seed"])
    X, info = c.solve(_dev(B), tol=w["tol"], j=0)
    assert info["status"] == "converged", info
    Xh = _host(X)
    Bm = op.block_to_mat(B)
    Xm = op.block_to_mat(Xh)
    assert np.max(true_residual(op.A_mat, Bm, Xm)) <= 1e-12
    assert np.max(info["true_residual"]) <= 1e-12
    Xd = np.linalg.solve(op.dense(), Bm)
    assert _rel(Xm, Xd) < 1e-10
    assert info["mvm_paper"] == 2 * info["iterations"] + 1 or info["restarts"] > 0
    # same iteration as the oracle's: iteration counts agree closely
    Xo, io = block_bicggr(op.A_mat, lambda m: m.copy(), Bm, w["tol"], 0)
    assert abs(io["iterations"] - info["iterations"]) <= 3
    c.close()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_solve_first_iterations_match_oracle(pkg, k):
    """After k outer iterations the GPU iterate equals the oracle's (same steps, FP64 rounding only)."""
    dims = (4, 4, 4, 6)
    U = wi.random_links(dims, 0.3, 120)
    op = WilsonClover(dims, U, 0.125, 1.4)
    c = _ctx(pkg, dims, U, 0.125, 1.4)
    B = wi.z4_block(op.V, 5, 121)
    for j in (0, 3):
        X, info = c.solve(_dev(B), tol=1e-30, j=j, max_iter=k, max_restarts=0)
        assert info["status"] == "not_converged" and info["iterations"] == k
        Bm = op.block_to_mat(B)
        from oracle.jacobi import jacobi_mat
        Xo, io = block_bicggr(op.A_mat, lambda m: jacobi_mat(op, m, j), Bm, 1e-30, j, max_iter=k)
        assert io["iterations"] == k
        assert _rel(op.block_to_mat(_host(X)), Xo) < 1e-12
        assert info["mvm_paper"] == io["mvm_paper"]
    c.close()


@pytest.mark.parametrize("L", [2, 7, 9, 13, 16])
def test_solve_every_block_width(pkg, L):
    """The fused update kernels are instantiated per block width: for widths the workloads do
    not use, the first two iterations equal the oracle's and a full solve reaches 1e-12 in the
    oracle's own true residual."""
    dims = (4, 4, 4, 6)
    U = wi.random_links(dims, 0.3, 122)
    op = WilsonClover(dims, U, 0.125, 1.4, bc_t=1)
    c = _ctx(pkg, dims, U, 0.125, 1.4, 1, max_L=16)
    B = wi.z4_block(op.V, L, 123 + L)
    Bm = op.block_to_mat(B)
    from oracle.jacobi import jacobi_mat
    X, info = c.solve(_dev(B), tol=1e-30, j=2, max_iter=2, max_restarts=0)
    Xo, io = block_bicggr(op.A_mat, lambda m: jacobi_mat(op, m, 2), Bm, 1e-30, 2, max_iter=2)
    assert info["iterations"] == io["iterations"] == 2
    assert _rel(op.block_to_mat(_host(X)), Xo) < 1e-12
    X, info = c.solve(_dev(B), tol=1e-12, j=2)
    assert info["status"] == "converged", info
    assert np.max(true_residual(op.A_mat, Bm, op.block_to_mat(_host(X)))) <= 1e-12
    c.close()


def test_solve_point_sources_jacobi_oracle_residual(pkg):
    """8^3 x 16, kappa 0.135, c_SW 1.6, twelve point sources, Jacobi j = 4, 8, 12, 16.  Here
    rho(kappa T^-1 H) = 1.047 > 1, so the longer Jacobi chains amplify rounding and a run may
    fail and be continued on halves of the block (splits); the cost formula of Table 1 is
    checked for the solves made of one run."""
    w, c, op = _workload_ctx(pkg, "lat8x16_L12_point")
    B = wi.point_block(op.V, 12)
    Bm = op.block_to_mat(B)
    for j in w["j"]:
        X, info = c.solve(_dev(B), tol=1e-12, j=j)
        assert info["status"] == "converged", info
        assert np.max(info["true_residual"]) <= 1e-12
        # independent check with the oracle's operator
        tr = true_residual(op.A_mat, Bm, op.block_to_mat(_host(X)))
        assert np.max(tr) <= 1e-12
        if info["restarts"] == 0 and info["splits"] == 0:
            assert info["mvm_paper"] == 2 * (j + 1) * info["iterations"] + 1
        _say(f"j={j}: k={info['iterations']} mvm/L={info['mvm_paper']} restarts={info['restarts']} "
             f"splits={info['splits']}")
    c.close()


def test_solve_failure_paths(pkg):
    dims = (4, 4, 4, 4)
    U = wi.random_links(dims, 0.3, 130)
    c = _ctx(pkg, dims, U, 0.12, 1.0)
    V = wi.volume(dims)
    b = wi.z4_block(V, 1, 131)
    X, info = c.solve(_dev(np.concatenate([b, b])), j=1, no_split=True)
    assert info["status"] == "breakdown" and info["splits"] == 0
    assert np.all(np.isfinite(_host(X)))
    Bz = wi.z4_block(V, 2, 132)
    Bz[1] = 0
    with pytest.raises(pkg.WDError):
        c.solve(_dev(Bz))
    X, info = c.solve(_dev(wi.z4_block(V, 2, 133)), j=0, max_iter=3, max_restarts=0)
    assert info["status"] == "not_converged" and info["iterations"] == 3
    X, info = c.solve(_dev(wi.z4_block(V, 2, 133)), j=0, diverge_at=1e-3, no_split=True, max_restarts=0)
    assert info["status"] == "diverged" and info["splits"] == 0
    # with splitting the halves diverge as well, and the solve says so
    X, info = c.solve(_dev(wi.z4_block(V, 2, 133)), j=0, diverge_at=1e-3, max_restarts=0)
    assert info["status"] == "diverged" and info["splits"] == 1 and info["min_block"] == 1
    c.close()


def test_solve_deterministic(pkg):
    dims = (4, 4, 4, 8)
    U = wi.random_links(dims, 0.3, 140)
    c = _ctx(pkg, dims, U, 0.13, 1.6)
    B = _dev(wi.point_block(wi.volume(dims), 6))
    X1, i1 = c.solve(B, j=4)
    X1 = _host(X1)
    X2, i2 = c.solve(B, j=4)
    assert np.array_equal(X1, _host(X2)) and i1["iterations"] == i2["iterations"]
    c.close()


# ---------------------------------------------------------------- full-size spot checks

@pytest.fixture(scope="module")
def big(pkg):
    """32^3 x 64 lattice with twelve columns: the bandwidth workload."""
    w = wi.workload("lat32x64_L12_point")
    U = wi.random_links(w["dims"], w["eps"], w["link_seed"])
    c = _ctx(pkg, w["dims"], U, w["kappa"], w["csw"], w["bc_t"], max_L=12)
    yield w, c, U
    c.close()


def _sample_sites(V, n=24, seed=7):
    rng = np.random.default_rng(seed)
    return sorted(set([0, V - 1] + list(rng.integers(0, V, n))))


def test_full_size_apply_sampled(pkg, big):
    w, c, U = big
    V = wi.volume(w["dims"])
    g = torch.Generator(device="cuda").manual_seed(5)
    X = torch.complex(torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64))
    Y = c.apply(X)
    so = SiteOperator(w["dims"], U, w["kappa"], w["csw"], w["bc_t"])
    sites = _sample_sites(V)
    need = sorted(set(sites) | {n for s in sites for (_, _, n, _) in so.neighbours(s)})
    idx = torch.tensor(need, device="cuda")
    Xs = X[:, :, idx].cpu().numpy()
    pos = {s: i for i, s in enumerate(need)}
    Ys = Y[:, :, torch.tensor(sites, device="cuda")].cpu().numpy()
    for k, s in enumerate(sites):
        ref = so.apply_at(s, lambda t: Xs[:, :, pos[t]].T)       # (12, L)
        assert _maxrel(Ys[:, :, k].T, ref) < 1e-13


def test_full_size_jacobi_two_sweeps_sampled(pkg, big):
    """Z = T^-1 (R + kappa H T^-1 R) at sampled sites (j = 2 reaches one hop)."""
    w, c, U = big
    V = wi.volume(w["dims"])
    g = torch.Generator(device="cuda").manual_seed(6)
    R = torch.complex(torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64))
    Z = c.jacobi(R, 2)
    so = SiteOperator(w["dims"], U, w["kappa"], w["csw"], w["bc_t"])
    sites = _sample_sites(V, 8, 9)
    need = sorted(set(sites) | {n for s in sites for (_, _, n, _) in so.neighbours(s)})
    Rs = R[:, :, torch.tensor(need, device="cuda")].cpu().numpy()
    pos = {s: i for i, s in enumerate(need)}
    Zs = Z[:, :, torch.tensor(sites, device="cuda")].cpu().numpy()
    Tinv = {s: np.linalg.inv(so.T(s)) for s in need}
    for k, s in enumerate(sites):
        g1 = lambda t: Tinv[t] @ Rs[:, :, pos[t]].T             # noqa: E731
        ref = Tinv[s] @ (Rs[:, :, pos[s]].T + w["kappa"] * so.hop_at(s, g1))
        assert _maxrel(Zs[:, :, k].T, ref) < 1e-13


@pytest.mark.parametrize("prec,tol", [("f32", 8e-6), ("bf16", 3e-2),
                                      ("f64c32", 9 * 2.0 ** -24), ("f64cbf16", 9 * 2.0 ** -8)])
def test_full_size_jacobi_two_sweeps_sampled_low_precision(pkg, big, prec, tol):
    """The low-precision Jacobi kernels in the benchmark's launch configuration (32^3 x 64,
    twelve columns), at sampled sites against the FP64 site operator, within twice the
    per-sweep bound derived for each storage format (rounded iterates: 1e3 u32 and 9 u_bf16
    per sweep; rounded coefficients only: 4.5 u)."""
    w, c, U = big
    V = wi.volume(w["dims"])
    g = torch.Generator(device="cuda").manual_seed(7)
    R = torch.complex(torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64))
    Z = c.jacobi(R, 2, prec=prec)
    so = SiteOperator(w["dims"], U, w["kappa"], w["csw"], w["bc_t"])
    sites = _sample_sites(V, 8, 10)
    need = sorted(set(sites) | {n for s in sites for (_, _, n, _) in so.neighbours(s)})
    Rs = R[:, :, torch.tensor(need, device="cuda")].cpu().numpy()
    pos = {s: i for i, s in enumerate(need)}
    Zs = Z[:, :, torch.tensor(sites, device="cuda")].cpu().numpy()
    del R, Z
    Tinv = {s: np.linalg.inv(so.T(s)) for s in need}
    ref, got = [], []
    for k, s in enumerate(sites):
        g1 = lambda t: Tinv[t] @ Rs[:, :, pos[t]].T             # noqa: E731
        ref.append(Tinv[s] @ (Rs[:, :, pos[s]].T + w["kappa"] * so.hop_at(s, g1)))
        got.append(Zs[:, :, k].T)
    err = _maxrel(np.stack(got), np.stack(ref))
    _say(f"full-size Jacobi j=2 {prec}: {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f64c32", 9 * 2.0 ** -24), ("f64cbf16", 9 * 2.0 ** -8)])
def test_full_size_jacobi_four_sweeps_sampled(pkg, big, prec, tol):
    """j = 4 in the benchmark's launch configuration (32^3 x 64, twelve columns): between the
    first and the last sweep the iterates are kept in the time-diagonal form (u + d, u - d), so
    this runs all three forms of the sweep, among them the middle sweep bench.py times.  The
    FP64 site operator recomputes G_k = T^-1 (R + kappa H G_{k-1}) on the dependence cone of the
    sampled sites (three hops for G_1, two for G_2, one for G_3); FP64 iterates with rounded
    coefficients are held to twice the per-sweep bound of their format (4.5 u)."""
    w, c, U = big
    V = wi.volume(w["dims"])
    g = torch.Generator(device="cuda").manual_seed(12)
    R = torch.complex(torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64))
    Z = c.jacobi(R, 4, prec=prec)
    so = SiteOperator(w["dims"], U, w["kappa"], w["csw"], w["bc_t"])
    sites = _sample_sites(V, 2, 11)
    cones = [set(sites)]
    for _ in range(3):
        cones.append(cones[-1] | {n for s in cones[-1] for (_, _, n, _) in so.neighbours(s)})
    need = sorted(cones[-1])
    Rs = R[:, :, torch.tensor(need, device="cuda")].cpu().numpy()
    pos = {s: i for i, s in enumerate(need)}
    Zs = Z[:, :, torch.tensor(sites, device="cuda")].cpu().numpy()
    del R, Z
    Tinv = {s: np.linalg.inv(so.T(s)) for s in need}
    G = {s: Tinv[s] @ Rs[:, :, pos[s]].T for s in need}          # G_1 on the three-hop cone
    for level in (2, 1, 0):
        G = {s: Tinv[s] @ (Rs[:, :, pos[s]].T + w["kappa"] * so.hop_at(s, lambda t: G[t])) for s in cones[level]}
    err = _maxrel(np.stack([Zs[:, :, k].T for k in range(len(sites))]), np.stack([G[s] for s in sites]))
    _say(f"full-size Jacobi j=4 {prec}: {err:.2e} at {len(sites)} sites ({len(need)} in the cone)")
    assert err < tol


def test_kappa_zero_is_identity(pkg):
    """kappa = 0: A = 1, A_D = 1 and the operator and every Jacobi application return their
    input bit for bit; the solver then converges in one iteration with X = B to rounding."""
    dims = (4, 4, 2, 6)
    U = wi.random_links(dims, 0.5, 150)
    c = _ctx(pkg, dims, U, 0.0, 1.7, 1)
    V = wi.volume(dims)
    Xd = _dev(wi.gaussian_block(V, 5, 151))
    assert torch.equal(c.apply(Xd), Xd)
    # j sweeps of G <- R + 0 * H G from G_0 = 0 with A_D = 1 give R exactly
    for j in (1, 2, 7):
        assert torch.equal(c.jacobi(Xd, j), Xd)
    X, info = c.solve(Xd, tol=1e-12, j=3)
    assert info["status"] == "converged" and info["iterations"] <= 1
    assert _maxrel(_host(X), _host(Xd)) < 1e-14          # the L x L coefficients are 1 up to rounding
    c.close()


@pytest.mark.parametrize("n,bc_t", [((0, 0, 0, 0), 0), ((1, 0, 2, 1), 0), ((3, 1, 1, 5), 0),
                                    ((0, 0, 0, 0), 1), ((2, 1, 0, 3), 1)])
def test_free_field_plane_wave(pkg, n, bc_t):
    """Unit links: A e^{ipx} u = [1 - 2 kappa sum cos p_mu + 2 i kappa sum gamma_mu sin p_mu] e^{ipx} u
    with p_mu = 2 pi n_mu / L_mu, and p_t = pi (2 n_t + 1) / L_t for antiperiodic time, checked on
    the GPU against the closed form."""
    from oracle import gammas
    dims = (4, 3, 4, 6)
    V = wi.volume(dims)
    kappa = 0.11
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[:, :] = np.eye(3)
    c = _ctx(pkg, dims, U, kappa, 1.3, bc_t)
    p = [2 * np.pi * n[m] / dims[m] for m in range(3)] + [np.pi * (2 * n[3] + bc_t) / dims[3]]
    s = np.arange(V)
    x = [s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2], s // (dims[0] * dims[1] * dims[2])]
    phase = np.exp(1j * sum(p[m] * x[m] for m in range(4)))            # (V,)
    rng = np.random.default_rng(152)
    u = rng.standard_normal((2, 12)) + 1j * rng.standard_normal((2, 12))  # two columns, row 3*spin + colour
    B = u[:, :, None] * phase[None, None, :]
    g = gammas()
    M4 = (1 - 2 * kappa * sum(np.cos(pm) for pm in p)) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
    M12 = np.kron(M4, np.eye(3))
    expect = (u @ M12.T)[:, :, None] * phase[None, None, :]
    Y = _host(c.apply(_dev(B)))
    assert _maxrel(Y, expect) < 1e-13
    c.close()


@pytest.mark.parametrize("bc_t", [0, 1])
def test_gauge_covariance_on_gpu(pkg, bc_t):
    """A[U^g](g psi) = g A[U] psi with U^g_mu(x) = g(x) U_mu(x) g(x + mu)^dag, both sides on the GPU
    (the links, clover and T^-1 are rebuilt from U^g), and the same for one Jacobi application."""
    dims = (4, 6, 2, 4)
    V = wi.volume(dims)
    lx, ly, lz, lt = dims
    U = wi.random_links(dims, 0.5, 160)
    gx = wi.random_gauge_transform(dims, 1.0, 161)
    s = np.arange(V)
    co = [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]
    Ug = np.empty_like(U)
    for mu in range(4):
        c = [a.copy() for a in co]
        c[mu] = (c[mu] + 1) % dims[mu]
        s2 = c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))
        Ug[mu] = gx @ U[mu] @ np.conj(np.transpose(gx[s2], (0, 2, 1)))
    c1 = _ctx(pkg, dims, U, 0.125, 1.3, bc_t)
    c2 = _ctx(pkg, dims, Ug, 0.125, 1.3, bc_t)
    psi = wi.gaussian_block(V, 3, 162)                                   # (L, 12, V)

    def gmul(b):                                                         # colour rotation per site
        f = b.reshape(b.shape[0], 4, 3, V)
        return np.einsum("vab,lsbv->lsav", gx, f).reshape(b.shape)

    lhs = _host(c2.apply(_dev(gmul(psi))))
    rhs = gmul(_host(c1.apply(_dev(psi))))
    assert _maxrel(lhs, rhs) < 1e-13
    lhs = _host(c2.jacobi(_dev(gmul(psi)), 4))
    rhs = gmul(_host(c1.jacobi(_dev(psi), 4)))
    assert _maxrel(lhs, rhs) < 1e-13
    c1.close()
    c2.close()


def test_single_link_clover_closed_form_on_gpu(pkg):
    """All links 1 except U_x(x0) = diag(e^{i phi}, e^{-i phi}, 1): the GPU clover equals the
    hand-derived T = 1 - kappa c_SW sigma_{x nu} F_{x nu}, F_{x nu} = +-(sin phi / 4) diag(1, -1, 0)
    at x0 +- nu and x0 + x +- nu, and 1 everywhere else (sigma_{x nu} = -diag(s3, s3),
    diag(s2, s2), diag(s1, -s1) for nu = y, z, t in the chiral basis)."""
    dims = (4, 4, 4, 4)
    V = wi.volume(dims)
    phi, kappa, csw = 0.7, 0.13, 1.9
    x0 = (1, 2, 1, 3)

    def site(c):
        c = [c[m] % dims[m] for m in range(4)]
        return c[0] + 4 * (c[1] + 4 * (c[2] + 4 * c[3]))

    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    U[0, site(x0)] = np.diag([np.exp(1j * phi), np.exp(-1j * phi), 1.0])
    c = _ctx(pkg, dims, U, kappa, csw, 0)
    T = c.clover(0)                                                      # (V, 2, 6, 6)
    c.close()
    f = np.sin(phi) / 4 * np.diag([1.0, -1.0, 0.0])
    s1 = np.array([[0, 1], [1, 0]])
    s2 = np.array([[0, -1j], [1j, 0]])
    s3 = np.array([[1, 0], [0, -1]])
    z2 = np.zeros((2, 2))
    sig = {1: -np.block([[s3, z2], [z2, s3]]), 2: np.block([[s2, z2], [z2, s2]]), 3: np.block([[s1, z2], [z2, -s1]])}
    expected = np.tile(np.eye(12, dtype=complex), (V, 1, 1))
    for nu in (1, 2, 3):
        for sign in (+1, -1):
            cc = list(x0)
            cc[nu] += sign
            for shift in (0, 1):
                c2 = list(cc)
                c2[0] += shift
                expected[site(c2)] -= kappa * csw * sign * np.kron(sig[nu], f)
    assert np.max(np.abs(expected[:, :6, 6:])) == 0 and np.max(np.abs(expected[:, 6:, :6])) == 0
    assert np.max(np.abs(T[:, 0] - expected[:, :6, :6])) < 1e-14
    assert np.max(np.abs(T[:, 1] - expected[:, 6:, 6:])) < 1e-14
