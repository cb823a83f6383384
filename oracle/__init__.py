"""Plain, slow FP64 CPU oracle for the LDG-Stokes multigrid V-cycle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check of
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.

The oracle is written from the paper (Saye, "Fast multigrid solution of
high-order accurate multi-phase Stokes problems"):

* ``basis``     orthonormal tensor-product Legendre basis, Gauss quadrature
* ``assemble``  fine-grid LDG operators by quadrature of the weak forms
                (appendix A: eq. geqn, ustarflux, sigmaresult, wform, ewv,
                Epenalty, stokessystem, viscousop)
* ``rhs``       right-hand side of eq. (stokessystem)
* ``coarsen``   operator coarsening, Algorithms 2 and 3 (appendix B)
* ``multigrid`` element-block Gauss-Seidel, Algorithm 1 (the V-cycle),
                eigen-decomposition bottom solver
* ``solvers``   stationary iteration, iterative refinement, FGMRES, the
                GMRES convergence metric of eq. (rho)
* ``errors``    error norms of the grid-convergence appendix

It shares no code with the HIP library.  All arithmetic is FP64 unless a
function says it emulates FP32.
"""
from .hierarchy import build_hierarchy, Hierarchy  # noqa: F401
