"""Conditioning of the synthetic ensembles on a 4^4 lattice, from the oracle's dense A:
the leftmost eigenvalue of A against kappa, the analogue of the paper's hopping
parameter next to its critical value (Sec. 3.1).  The unpreconditioned 4^4
workload (kappa 0.12, c_SW 1.0) must be subcritical (its dense-LU parity solve
converges); with c_SW 1.6 the leftmost eigenvalue moves left with kappa and has
crossed zero by 0.135 on this small volume.  Measured values are written to
WDSOLVE_RESULTS_DIR when that is set."""

import json
import os

import numpy as np

import wdinputs as wi
from oracle import WilsonClover


def _spectrum(dims, eps, seed, kappa, csw):
    op = WilsonClover(dims, wi.random_links(dims, eps, seed), kappa, csw)
    ev = np.linalg.eigvals(op.dense())
    return float(ev.real.min()), float(np.abs(ev).min())


def test_leftmost_eigenvalue_against_kappa():
    dims = (4, 4, 4, 4)
    c0 = _spectrum(dims, 0.3, 1001, 0.12, 1.0)           # the 4^4 dense-LU workload
    c2a = _spectrum(dims, 0.3, 1003, 0.127, 1.6)         # eps and c_SW of the 16^3 x 32 runs
    c2b = _spectrum(dims, 0.3, 1003, 0.135, 1.6)
    rec = {"c0_kappa0.12": c0, "eps0.3_csw1.6_kappa0.127": c2a, "eps0.3_csw1.6_kappa0.135": c2b}
    out = os.environ.get("WDSOLVE_RESULTS_DIR")
    if out and os.path.isdir(out):
        with open(os.path.join(out, "conditioning_4x4.json"), "w") as f:
            json.dump({k: {"min_re": v[0], "min_abs": v[1]} for k, v in rec.items()}, f, indent=1)
    assert c0[0] > 0.05 and c0[1] > 0.05
    assert c2a[0] > c2b[0]
    assert c2b[0] < 0.0
