"""Named synthetic workloads (lattice, link ensemble, operator parameters, sources, solver settings).

They stand in for the paper's test problem (Sec. 3.1: 16^3 x 32 lattice,
quenched configurations, point sources, Sec. 3.3), which cannot be
reproduced without its gauge ensemble.  kappa and c_SW differ from the
paper's because random links have a different critical kappa.
"""

from __future__ import annotations

WORKLOADS = {
    # 4^4 lattice, N = 3072: small enough for a dense LU cross-check.
    "lat4_L4_z4": dict(
        dims=(4, 4, 4, 4), eps=0.3, link_seed=1001, kappa=0.12, csw=1.0,
        L=4, source="z4", source_seed=2001, j=(0,), tol=1e-12, bc_t=0,
    ),
    # 8^3 x 16 lattice, twelve point sources, Jacobi j in {4, 8, 12, 16}.
    "lat8x16_L12_point": dict(
        dims=(8, 8, 8, 16), eps=0.3, link_seed=1002, kappa=0.135, csw=1.6,
        L=12, source="point", source_seed=0, j=(4, 8, 12, 16), tol=1e-12, bc_t=0,
    ),
    # The paper's lattice size, 16^3 x 32, L sweep at j = 12 (kappa = 0.135
    # stagnates near 1e-9 on this ensemble; 0.130 converges).
    "lat16x32_point": dict(
        dims=(16, 16, 16, 32), eps=0.3, link_seed=1003, kappa=(0.130, 0.135), kappa_solve=0.130, csw=1.6,
        L=(1, 2, 3, 4, 6, 12), source="point", source_seed=0, j=(12,), tol=1e-12, bc_t=0,
    ),
    # 32^3 x 64 lattice (N = 25.2M), twelve point sources: the bandwidth headline.
    # kappa = 0.135 lies past the critical hopping parameter of this ensemble
    # (A has eigenvalues with negative real part and the solve does not
    # converge), so solves use kappa_solve = 0.127, just below it.
    "lat32x64_L12_point": dict(
        dims=(32, 32, 32, 64), eps=0.2, link_seed=1004, kappa=0.135, kappa_solve=0.127, csw=1.6,
        L=12, source="point", source_seed=0, j=(12,), tol=1e-12, bc_t=0,
    ),
}


def workload(name: str) -> dict:
    w = dict(WORKLOADS[name])
    w["name"] = name
    return w
