"""FP64 CPU oracle for the Jacobi-preconditioned block BiCGGR hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C ABI library
and its Python binding) imports, links or calls this package.  Only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.

It is plain numpy in float64/complex128 (float32 where ``lowp`` emulates a
storage format), written for obvious correctness,
not speed, and it shares no code, tables or constants with the HIP path.
It works in its own array layout (fields shaped ``(Lt, Lz, Ly, Lx, 4, 3, L)``:
t, z, y, x, spin, colour, column) and converts from/to the exchange layout
of the C ABI at its edges.

Contents (each function cites the passage it follows):

* ``dirac``   -- gamma matrices, clover field strength, the site matrix T,
                 the hopping term H and the clover Wilson-Dirac operator
                 A = T - kappa H; dense assembly of A for small lattices.
* ``jacobi``  -- the Jacobi preconditioner M (Sec. 2, the display after the
                 algorithm box), written as the paper's closed-form sum.
* ``bbicggr`` -- preconditioned block BiCGGR (Sec. 2, algorithm box), step
                 by step, with the stopping rule of Sec. 3.3.
* ``bicgstab`` -- preconditioned block BiCGSTAB (the published block
                 version of BiCGSTAB), the foil whose recursive residual drifts
                 from the true one, which BiCGGR is built to avoid (Sec. 1).
* ``lowp``    -- the low-precision storage of the Jacobi preconditioner
                 and operator: FP32 / BF16 (round-to-nearest-even) rounding of
                 the links (two stored rows, the third rebuilt), the site
                 matrices, inputs and stored iterates, with float32
                 arithmetic.
* ``learned`` -- the linear gauge-covariant network layers used as an
                 alternative preconditioner: forward, adjoint, the error and
                 residual losses with their gradients, Adam.

The operator itself is not printed in the paper (Sec. 2 defers it to the
companion application paper); the convention used here is the standard
hopping-parameter form of the O(a)-improved Wilson-Dirac matrix, stated in
``dirac`` and pinned by closed forms (free-field plane waves, a single-link
clover field), gamma5-hermiticity, gauge covariance and dense-matrix checks.
"""

from . import dirac, jacobi, bbicggr, bicgstab  # noqa: F401
from .dirac import WilsonClover, gammas, gamma5, sigma_munu  # noqa: F401
from .jacobi import jacobi_apply  # noqa: F401
from .bbicggr import block_bicggr, solve_with_restarts  # noqa: F401
from .bicgstab import block_bicgstab  # noqa: F401
