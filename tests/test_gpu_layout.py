"""The tiled layout of block vectors (wd_set_layout), through the C ABI.

In the tiled layout row n of a column is (s // 64) * 768 + k * 64 + s % 64 instead
of k * V + s: the same matrices in another memory order.  Every kernel computes
each site with the same arithmetic in the same order in either layout, so results
must agree with the standard layout bit for bit, and with the FP64 oracle to the
usual 1e-13.  The solver runs in the tiled layout for a caller of the standard one
(copying B and X in and X out), which the bit-equal solve below checks as well; so
do the learned preconditioner's layers, gradient and training.
"""

import sys

import numpy as np
import pytest

import wdinputs as wi
from oracle import WilsonClover
from oracle.jacobi import jacobi_apply

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


def tiled(b):
    """(L, 12, V) standard-layout array -> the same matrix in the tiled memory order."""
    L, _, V = b.shape
    return b.reshape(L, 12, V // 64, 64).transpose(0, 2, 1, 3).reshape(L, 12, V)


def untiled(b):
    L, _, V = b.shape
    return b.reshape(L, V // 64, 12, 64).transpose(0, 2, 1, 3).reshape(L, 12, V)


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


def _maxrel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def test_layout_helpers_are_inverse():
    b = np.arange(2 * 12 * 128).reshape(2, 12, 128)
    t = tiled(b)
    assert np.array_equal(untiled(t), b)
    # column 1, k = 5, site 70: row (70 // 64) * 768 + 5 * 64 + 70 % 64 of column 1
    flat = np.ascontiguousarray(t).reshape(-1)
    assert flat[12 * 128 + 1 * 768 + 5 * 64 + 6] == b[1, 5, 70]


@pytest.mark.parametrize("dims", [(3, 3, 3, 3), (2, 2, 2, 2), (5, 3, 3, 5)])
def test_tiled_layout_needs_whole_tiles(pkg, dims):
    c = pkg.Context(dims, max_L=2)
    with pytest.raises(pkg.WDError):
        c.set_layout("tiled")
    c.close()


# Lattices with V a multiple of 64 over the site maps of the stencils: (4, 4, 4, 4) the 2 x 4
# split with one z plane per XCD, (8, 16, 8, 3) the 1 x 8 split, (16, 8, 4, 4) the rows map of
# the LDS-staged kernels, (8, 6, 4, 10) uneven tiles per plane.
DIMS = [((4, 4, 4, 4), 0), ((8, 16, 8, 3), 1), ((16, 8, 4, 4), 1), ((8, 6, 4, 10), 0)]


@pytest.mark.parametrize("dims,bc_t", DIMS)
@pytest.mark.parametrize("L", [1, 2, 5, 12])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_apply_tiled_equals_standard(pkg, dims, bc_t, L, prec):
    """L = 1, 2: the register-tiled kernel; 5, 12: the LDS-staged one (FP64 and FP32)."""
    U = wi.random_links(dims, 0.4, 202)
    c = _ctx(pkg, dims, U, 0.128, 1.6, bc_t)
    V = wi.volume(dims)
    X = wi.gaussian_block(V, L, 203)
    Ys = _host(c.apply(_dev(X), prec=prec))
    c.set_layout("tiled")
    Yt = untiled(_host(c.apply(_dev(tiled(X)), prec=prec)))
    assert np.array_equal(Yt, Ys)
    if prec == "f64":
        op = WilsonClover(dims, U, 0.128, 1.6, bc_t=bc_t)
        assert _maxrel(Yt, op.to_block(op.apply_A(op.from_block(X)))) < 1e-13
    c.close()


@pytest.mark.parametrize("L", [2, 3, 7])
@pytest.mark.parametrize("j", [1, 2, 5])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("prec", ["f64", "f64c32", "f64cbf16", "f32", "bf16"])
def test_jacobi_tiled_equals_standard(pkg, L, j, kind, prec):
    """Every Jacobi path: first sweep, register-tiled (L = 2) and LDS-staged sweeps, FP64
    iterates in the time-diagonal form between sweeps (L >= 3, j >= 3), rounded coefficients,
    FP32 and BF16 iterates."""
    dims = (4, 4, 6, 4)
    U = wi.random_links(dims, 0.3, 209)
    c = _ctx(pkg, dims, U, 0.13, 1.6, 1, kind=kind)
    V = wi.volume(dims)
    R = wi.gaussian_block(V, L, 210)
    Zs = _host(c.jacobi(_dev(R), j, prec=prec))
    c.set_layout("tiled")
    Zt = untiled(_host(c.jacobi(_dev(tiled(R)), j, prec=prec)))
    assert np.array_equal(Zt, Zs)
    if prec == "f64":
        op = WilsonClover(dims, U, 0.13, 1.6, bc_t=1, jacobi_kind="block" if kind == 0 else "point")
        assert _maxrel(Zt, op.to_block(jacobi_apply(op, op.from_block(R), j))) < 1e-13
    c.close()


@pytest.mark.parametrize("prec", ["f64", "f64c32", "f64cbf16"])
def test_hop_repeat_tiled_equals_standard(pkg, prec):
    dims = (8, 16, 8, 3)
    U = wi.random_links(dims, 0.3, 211)
    c = _ctx(pkg, dims, U, 0.13, 1.6, 1)
    V = wi.volume(dims)
    X = wi.gaussian_block(V, 12, 212)
    R = wi.gaussian_block(V, 12, 213)
    out = {}
    for layout in ("standard", "tiled"):
        c.set_layout(layout)
        f = tiled if layout == "tiled" else (lambda b: b)
        g = untiled if layout == "tiled" else (lambda b: b)
        Y = c.empty_block(12)
        c.hop_repeat(_dev(f(X)), Y, 2, mode=1, R=_dev(f(R)), prec=prec)
        out[layout] = [g(_host(Y))]
        if prec == "f64":
            c.hop_repeat(_dev(f(X)), Y, 1, mode=0)
            out[layout].append(g(_host(Y)))
    for a, b in zip(out["standard"], out["tiled"]):
        assert np.array_equal(a, b)
    c.close()


def test_solve_in_tiled_context_equals_standard_caller(pkg):
    """A standard-layout caller's solve runs in the tiled layout (B and X copied in, X out): the
    same arithmetic as a solve on a tiled context, so X agrees bit for bit, with and without an
    initial guess; snapshots are copied out in the caller's layout and do not change the solve."""
    dims = (4, 4, 4, 6)
    U = wi.random_links(dims, 0.3, 214)
    op = WilsonClover(dims, U, 0.125, 1.4, bc_t=1)
    V = wi.volume(dims)
    B = wi.z4_block(V, 5, 215)
    X0 = 0.1 * wi.gaussian_block(V, 5, 216)
    cs = _ctx(pkg, dims, U, 0.125, 1.4, 1)
    ct = _ctx(pkg, dims, U, 0.125, 1.4, 1)
    ct.set_layout("tiled")
    for x0 in (None, X0):
        Xs, infs = cs.solve(_dev(B), None if x0 is None else _dev(x0), tol=1e-12, j=3)
        Xt, inft = ct.solve(_dev(tiled(B)), None if x0 is None else _dev(tiled(x0)), tol=1e-12, j=3)
        assert infs["status"] == inft["status"] == "converged"
        assert infs["iterations"] == inft["iterations"]
        assert np.array_equal(untiled(_host(Xt)), _host(Xs))
        assert list(infs["true_residual"]) == list(inft["true_residual"])
    snap = torch.empty((10, 12, V), dtype=torch.complex128, device="cuda")
    Xn, infn = cs.solve(_dev(B), tol=1e-12, j=3, x_snap=snap, snap_every=3)
    Xs, infs = cs.solve(_dev(B), tol=1e-12, j=3)
    assert infn["status"] == "converged" and infn["snapshots"] == 2
    assert torch.equal(Xn, Xs)
    for i in (1, 2):
        Xk, _ = cs.solve(_dev(B), tol=1e-30, j=3, max_iter=3 * i, max_restarts=0)
        assert torch.equal(snap[5 * (i - 1):5 * i], Xk)
    from oracle.bbicggr import true_residual
    assert np.max(true_residual(op.A_mat, op.block_to_mat(B), op.block_to_mat(_host(Xs)))) <= 1e-12
    cs.close()
    ct.close()


@pytest.mark.parametrize("L", [2, 3, 12])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_learned_apply_tiled_equals_standard(pkg, L, prec):
    """The learned layers (FP64: LDS-staged from three columns on; FP32: column tiles)."""
    dims = (8, 16, 8, 3)
    U = wi.random_links(dims, 0.3, 217)
    c = _ctx(pkg, dims, U, 0.12, 1.0)
    c.learned_init("neumann")
    V = wi.volume(dims)
    R = wi.gaussian_block(V, L, 218)
    Zs = _host(c.learned_apply(_dev(R), prec=prec))
    c.set_layout("tiled")
    Zt = untiled(_host(c.learned_apply(_dev(tiled(R)), prec=prec)))
    assert np.array_equal(Zt, Zs)
    c.close()


@pytest.mark.parametrize("loss", ["error", "residual"])
def test_learned_gradient_and_training_tiled_equal_standard(pkg, loss):
    """The weight gradient sums over sites in the same order in both layouts, so it agrees bit
    for bit; the loss sums over elements in memory order and agrees to rounding; three Adam
    steps then give the same weights."""
    dims = (4, 4, 4, 8)
    U = wi.random_links(dims, 0.3, 219)
    V = wi.volume(dims)
    R = wi.gaussian_block(V, 3, 220)
    E = wi.gaussian_block(V, 3, 221)
    Rp = wi.gaussian_block(V, 6, 222)
    Ep = wi.gaussian_block(V, 6, 223)
    res = {}
    for layout in ("standard", "tiled"):
        f = tiled if layout == "tiled" else (lambda b: b)
        c = _ctx(pkg, dims, U, 0.12, 1.0)
        c.set_layout(layout)
        c.learned_init("neumann")
        lv, G = c.learned_grad(_dev(f(R)), _dev(f(E)) if loss == "error" else None, loss=loss)
        c.learned_train(_dev(f(Rp)), _dev(f(Ep)) if loss == "error" else None, L=3, steps=3, loss=loss)
        res[layout] = (lv, G, c.get_learned())
        c.close()
    (ls_, Gs, ths), (lt, Gt, tht) = res["standard"], res["tiled"]
    assert abs(lt - ls_) <= 1e-12 * abs(ls_)
    assert np.array_equal(Gt, Gs)
    assert np.array_equal(tht, ths)


def test_full_size_jacobi_tiled_equals_standard(pkg):
    """The benchmark's launch configuration (32^3 x 64, twelve columns, j = 4: first sweep, the
    three forms of the time-diagonal sweep), the tiled layout against the standard one over the
    whole output."""
    w = wi.workload("lat32x64_L12_point")
    U = wi.random_links(w["dims"], w["eps"], w["link_seed"])
    c = _ctx(pkg, w["dims"], U, w["kappa"], w["csw"], w["bc_t"])
    V = wi.volume(w["dims"])
    g = torch.Generator(device="cuda").manual_seed(13)
    R = torch.complex(torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((12, 12, V), generator=g, device="cuda", dtype=torch.float64))
    Zs = c.jacobi(R, 4)
    Ys = c.apply(R)
    Rt = R.reshape(12, 12, V // 64, 64).permute(0, 2, 1, 3).contiguous()
    del R
    c.set_layout("tiled")
    Zt = c.jacobi(Rt.view(12, 12, V), 4)
    assert torch.equal(Zt.view(12, V // 64, 12, 64).permute(0, 2, 1, 3).reshape(12, 12, V), Zs)
    del Zt, Zs
    Yt = c.apply(Rt.view(12, 12, V))
    assert torch.equal(Yt.view(12, V // 64, 12, 64).permute(0, 2, 1, 3).reshape(12, 12, V), Ys)
    c.close()
