"""Plain FP64 CPU oracle for the generalized Stokes solve (TEST INFRASTRUCTURE ONLY).

This package is the independent reference that the GPU library is checked
against.  It is slow and obvious on purpose: NumPy/SciPy in float64, no
blocking, no fusion, no reordering beyond what the definitions state.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (``paper_2407_01783_amd``) never
imports, calls or links anything here, and this package imports nothing from
the product path: the two share no code, tables or constants.

What it computes (Creff & Guermond, "Preconditioning of the generalized Stokes
problem ...", arXiv 2407.01783):

* ``mesh``   -- the structured Kuhn simplex mesh of the unit square / cube, the
  P2 (velocity) and P1 (pressure) node numbering and the seeded vertex jitter.
* ``fem``    -- element matrices by exact barycentric integration and global
  assembly of M_V, L_V, B, M_Q, L_Q and the lumped Lambda_V (Sec. 2.2,
  Sec. 3.2, Sec. 4.1).
* ``p3``     -- the Taylor-Hood P3/P2 pair on the same Kuhn mesh (the paper's
  second element pair, Sec. 3.3, Table 4): P3 numbering on the (3n+1)^d
  lattice, exact P3/P2 reference integrals, closed-form int |phi_i|, and the
  assembly; ``stokes`` solves with these matrices unchanged.
* ``stokes`` -- Dirichlet elimination and lifting, the saddle-point system
  A U - B^T P = F, B U = g (Sec. 2.2, Eq. "Saddle_point_A_BT_B"), its direct or
  MINRES solution with the pressure normalised to zero mean, the true coupled
  residual, and the adjoint gradient of a quadratic loss.

Every function names the passage of the paper it follows.  Readings of points
where the paper is silent or garbled are listed in the repository's design
notes; the ones that matter here are repeated in the docstrings.
"""

from . import mesh, fem, stokes, p3  # noqa: F401
