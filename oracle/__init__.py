"""FP64 CPU oracle for the space-time isogeometric Galerkin heat-equation solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_1909_07309_amd``); the only module both sides import is
``workloads`` (seeded random draws and sizes, none of the method's arithmetic).

Everything here is plain numpy/scipy in float64, written from the paper
(Loli, Montardini, Sangalli, Tani, "An efficient solver for space-time
isogeometric Galerkin methods for parabolic problems", arXiv:1909.07309):

* ``bsplines``  - knot vectors, Cox-de Boor recursion (Section 2.1), 1D
                  Galerkin matrices W_t, M_t, K_l, M_l (eq. time_mat,
                  space_univ_par_mat), Gauss-Legendre quadrature.
* ``dense``     - dense Kronecker assembly of A and A-hat (eq. syst_mat,
                  prec_definition), an independent brute-force space-time
                  quadrature of the bilinear form (Section 3.1), direct solves.
* ``fd``        - the fast-diagonalization apply of A-hat^{-1} with banded
                  shifted time solves, and a Kronecker matvec (Section 4.4,
                  Section 4.5), for full-size checks and the CPU baseline.
* ``arrowhead`` - the paper's stable arrowhead factorization of the time
                  pencil and Algorithm 1 with the block-LU middle solve
                  (Sections 4.2-4.4), as an independent cross-check of ``fd``.
* ``annulus``   - quarter-annulus geometry, variable separable coefficients,
                  the geometry-aware preconditioner A-hat^G (Section 4.3).
* ``annulus3d`` - the same on the quarter annulus extruded to 3D, with the
                  3D separation of the coefficients (Section 4.3 in 3D).
* ``convergence`` - errors of manufactured solutions (Section 5.1 rates): on
                  the unit square and cube, and on the quarter annulus with the
                  annulus workload's variable conductivity and heat capacity,
                  which pins that workload's assembly.
* ``adjoint``   - dense adjoint gradients of a quadratic loss.
* ``problems``  - load vectors of the synthetic workloads.

Functions without an independent pin say "parity unpinned" in their docstring.
The variable-coefficient assembly of ``annulus`` is pinned by the manufactured
rates and by an exact Kronecker form for a polar-separable conductivity; the 3D
assembly of ``annulus3d`` by the exact Kronecker form for a conductivity
separable in (r, theta, z) and by sharing the pinned 1/c-weighted time factor.
"""
