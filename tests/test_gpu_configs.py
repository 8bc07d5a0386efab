"""Solves on the paper's lattice size, 16^3 x 32 with point sources (Sec. 3.1,
3.3), for L = 1 .. 12 right-hand sides, through the C ABI.

Each solve must reach a true residual <= 1e-12 per column, recomputed with
the oracle's operator on the whole lattice; a run that loses rank and fails
is continued on the halves of its block.  Without restarts or splits the cost count
must equal 2(j+1)k + 1 applications per column, the relation every entry of
Table 1 satisfies.  Iteration counts on these synthetic links are recorded
(the paper's numbers need its gauge ensemble, so they are not compared).
"""

import json
import os
import sys

import numpy as np
import pytest

import wdinputs as wi
from oracle import WilsonClover
from oracle.bbicggr import true_residual

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_REC = {}


def _say(msg):
    sys.__stderr__.write(f"[configs] {msg}\n")
    sys.__stderr__.flush()


def _record(key, val):
    _REC[key] = val
    out = os.environ.get("WDSOLVE_RESULTS_DIR")      # optional: keep the measured values as JSON
    if out and os.path.isdir(out):
        with open(os.path.join(out, "lsweep.json"), "w") as f:
            json.dump(_REC, f, indent=1)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0907_3261_amd as pkg
    pkg.load()
    w = wi.workload("lat16x32_point")
    U = wi.random_links(w["dims"], w["eps"], w["link_seed"])
    kappa = w["kappa_solve"]
    c = pkg.Context(w["dims"], bc_t=w["bc_t"], max_L=12)
    c.set_links(U)
    c.set_params(kappa, w["csw"])
    op = WilsonClover(w["dims"], U, kappa, w["csw"], bc_t=w["bc_t"])
    yield pkg, c, op, w
    c.close()


@pytest.mark.parametrize("L", [1, 2, 3, 4, 6, 12])
def test_point_source_solve_l_sweep(setup, L):
    pkg, c, op, w = setup
    j = 12
    B = wi.point_block(op.V, L)
    _say(f"L={L} j={j}")
    # few right-hand sides converge slowly here, with plateaus of hundreds of iterations
    X, info = c.solve(torch.from_numpy(B).cuda(), tol=1e-12, j=j, stagnate_window=3000, max_iter=20000)
    _say(f"L={L}: {info['status']} k={info['iterations']} restarts={info['restarts']}")
    _record(f"L{L}", {"status": info["status"], "iterations": info["iterations"], "restarts": info["restarts"],
                      "total_iterations": info["total_iterations"], "splits": info["splits"],
                      "min_block": info["min_block"], "cond_max": info["cond_max"],
                      "mvm_paper_per_col": int(info["mvm_paper"]), "s_per_rhs": info["seconds"] / L})
    # with one to three sources this ensemble sits close to the critical kappa and a block run can
    # lose rank and diverge (the paper's Table 1 has such failures too); the driver then solves
    # the halves of the block on their own (Sec. 3.3), so every width must converge
    assert info["status"] == "converged", info
    tr = true_residual(op.A_mat, op.block_to_mat(B), op.block_to_mat(X.cpu().numpy()))
    assert np.max(tr) <= 1e-12
    np.testing.assert_allclose(info["true_residual"][:L], tr, rtol=0.05, atol=1e-15)  # both are rounding-limited
    if info["restarts"] == 0 and info["splits"] == 0:
        assert info["mvm_paper"] == 2 * (j + 1) * info["iterations"] + 1
    _REC[f"L{L}"]["true_residual_max"] = float(np.max(tr))
    _record(f"L{L}", _REC[f"L{L}"])


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_low_precision_jacobi_solve_l12(setup, prec):
    pkg, c, op, w = setup
    B = wi.point_block(op.V, 12)
    X, info = c.solve(torch.from_numpy(B).cuda(), tol=1e-12, j=12, prec_inner=prec)
    assert info["status"] == "converged", info
    tr = true_residual(op.A_mat, op.block_to_mat(B), op.block_to_mat(X.cpu().numpy()))
    assert np.max(tr) <= 1e-12
    _record(f"L12_{prec}", {"iterations": info["total_iterations"], "cycles": info["cycles"],
                            "fallback": info["fallback"], "s_per_rhs": info["seconds"] / 12,
                            "true_residual_max": float(np.max(tr))})


def test_point_source_solve_at_nominal_kappa(pkg_kappa135):
    """The configuration's nominal kappa 0.135 (rho(kappa T^-1 H) = 1.045 on this ensemble): twelve
    point sources, FP64 Jacobi j = 12.  The full block loses rank (its condition estimate climbs
    before the run fails) and the driver finishes it on the halves of the block (Sec. 3.3), which
    reach the 1e-12 true residual."""
    pkg, c, op, w = pkg_kappa135
    L = 12
    B = wi.point_block(op.V, L)
    X, info = c.solve(torch.from_numpy(B).cuda(), tol=1e-12, j=12, max_iter=3000)
    _say(f"kappa 0.135 L={L}: {info['status']} k={info['total_iterations']} splits={info['splits']} "
         f"min_block={info['min_block']} cond_max={info['cond_max']:.2e}")
    _record("L12_kappa0.135", {"status": info["status"], "total_iterations": info["total_iterations"],
                               "splits": info["splits"], "min_block": info["min_block"],
                               "cond_max": info["cond_max"], "s_per_rhs": info["seconds"] / L})
    assert info["status"] == "converged", info
    tr = true_residual(op.A_mat, op.block_to_mat(B), op.block_to_mat(X.cpu().numpy()))
    assert np.max(tr) <= 1e-12


@pytest.fixture(scope="module")
def pkg_kappa135():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0907_3261_amd as pkg
    pkg.load()
    w = wi.workload("lat16x32_point")
    U = wi.random_links(w["dims"], w["eps"], w["link_seed"])
    c = pkg.Context(w["dims"], bc_t=w["bc_t"], max_L=12)
    c.set_links(U)
    c.set_params(0.135, w["csw"])
    op = WilsonClover(w["dims"], U, 0.135, w["csw"], bc_t=w["bc_t"])
    yield pkg, c, op, w
    c.close()
