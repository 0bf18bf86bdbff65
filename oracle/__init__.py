"""Plain FP64 CPU oracle for the immersed-boundary acoustic finite-difference method
of Caunt, Nelson, Luporini and Gorman, "A Novel Immersed Boundary Approach for
Irregular Topography with Acoustic Wave Equations" (arXiv 2309.03600).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or call it.  The HIP
library and its Python binding never import it, and it imports nothing from them.

Every function is written from the paper's mathematics (sections and equations are
cited in each docstring) as slowly and plainly as practical: per-point Python loops,
``numpy.linalg`` SVD / pseudoinverse, ``scipy.sparse`` matrices.  No blocking, fusion
or reordering beyond what the definitions state.

Modules
-------
basis      multi-indices, Taylor rows, boundary-condition operator rows
fd         textbook centred / staggered finite-difference weights (Fornberg)
geometry   heightfield surface, foot points, classification, eta exclusion
weights    immersed-boundary points, per-point systems, rank rule, modified stencils
stepper    sparse modified Laplacian and the damped leapfrog time stepper
analytic   method-of-images solutions for flat free / rigid surfaces
adjoint    discrete adjoint of the stepper and the velocity gradient
staggered  first-order pressure-velocity form on a staggered grid
mulder1d   per-axis 1D extrapolation (the reduction to 1D)
forcing    inhomogeneous boundary conditions (the forcing columns of B A^+)
           (the mixed surface p + a(x_b) dp/dn = 0 lives in basis and weights)

Parity status: every function is pinned by tests under ``tests/test_oracle_*.py``
except where a docstring says "parity unpinned".
"""
