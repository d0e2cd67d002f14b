"""CPU FP64 oracle for the V-FPI contact solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls it and shares no code with it; the only code
both sides use is the seeded input generator package ``scenes``.

Everything is plain NumPy/SciPy in float64, written from the paper
("Large-Dimensional Multibody Dynamics Simulation Using Contact Nodalization
and Diagonalization", Lee, Lee & Lee):

* ``core``       -- the problem definition (A, J_c), the step-size matrix W
                    (Sec. IV-C), the surrogate Delassus operator (Prop. 3), the
                    strict and proximal projections (eq. operator) and the V-FPI
                    loop itself (Alg. 1 with Alg. 2 as its contact step).
* ``delassus``   -- the original problem solved the classical way: projected
                    Gauss-Seidel on the Delassus operator (eq. delassus; the
                    paper's I-FPI baseline), with the Cholesky factor of A.
* ``enumerate``  -- brute-force contact-mode enumeration on the Delassus form.
* ``adjoint``    -- implicit differentiation of the converged V-FPI step.
* ``batched``    -- independent environments solved one after another.
* ``chebyshev``  -- V-FPI with Chebyshev acceleration (Alg. 3).

Each function names the passage it follows.  Parity pins: see the module
headers; "parity unpinned" is stated where no independent pin exists.
"""
from .core import (BRANCH_OPEN, BRANCH_SLIP, BRANCH_STICK, contact_jacobian, frobenius_w,
                   project_proximal, project_strict, row_stats, surrogate_delassus,
                   system_matrix, validate, vfpi)

__all__ = [
    "BRANCH_OPEN", "BRANCH_STICK", "BRANCH_SLIP", "contact_jacobian", "frobenius_w",
    "project_proximal", "project_strict", "row_stats", "surrogate_delassus",
    "system_matrix", "validate", "vfpi",
]
