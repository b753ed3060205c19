"""MI355X (gfx950) generalized Stokes solver: Taylor-Hood P2/P1 on Kuhn meshes,
Schur-complement CG with Cahouet-Chabard preconditioning and block-preconditioned
flexible GMRES on the coupled system, behind the C ABI of include/stokes.h.

Importing the package does not load the library; ``_lib.load()`` (called by
``StokesProblem``) does, and fails when libstokes.so has not been built.
"""

from . import inputs  # noqa: F401

__all__ = ["inputs", "StokesProblem", "StokesSolve"]


def __getattr__(name):
    if name in ("StokesProblem", "StokesSolve"):
        from . import stokes
        return getattr(stokes, name)
    raise AttributeError(name)
