"""CPU oracle for the stage-parallel Radau IIA heat-equation solver.

This package is TEST INFRASTRUCTURE ONLY.  It is a plain, slow, obviously
correct fp64 implementation of what the GPU library computes, written from
the paper (Munch, Dravins, Kronbichler, Neytcheva, "Stage-parallel fully
implicit Runge-Kutta implementations with optimal multilevel preconditioners
at the scaling limit", arXiv:2209.06700).  Only ``tests/``, the
``__graft_entry__.smoke()`` check and the ``cpu_baseline`` leg of ``bench.py``
may import it.  The product path (``paper_2209_06700_amd``) never imports,
calls or links anything here, and this package never imports the product.

Modules
-------
tableau    Radau IIA Butcher tableau, A^-1, its Crout factor L and the
           eigen-decomposition L = S Lambda S^-1 (Sec. 2, eq. irk:P).
fe         1D Q_k Lagrange elements on Gauss-Lobatto nodes, Gauss quadrature,
           element matrices, nested-space prolongation (Sec. 5 set-up).
assemble   cell-loop assembly of the global mass/stiffness matrices on the
           n^3 uniform hexahedral mesh of the unit cube, loads, interpolation.
step       the Radau IIA step: direct sparse solve of the stage system
           (Sec. 2), backward Euler, and the exact modal solve.
multigrid  Chebyshev-Jacobi smoother, geometric multigrid V-cycle and the
           stage-block preconditioner P^-1 (eq. irk:P, Sec. 5).
fgmres     right-preconditioned flexible GMRES on the premultiplied stage
           operator (eq. irk:A).
complex_irk  direct diagonalisation A_Q^-1 = S Lam S^-1 (eq. irk:Ainv) in
           real two-by-two form, the PRESB preconditioner (Sec. 6) and the
           step that solves every block with its own GMRES.
pointwise  single rows of the assembled operators, for sampled checks on
           meshes too large to assemble.
deformed   mass and stiffness matrices on a smoothly deformed (non-affine)
           hexahedral mesh with per-quadrature-point Jacobians, and sampled
           rows for meshes too large to assemble.
"""
