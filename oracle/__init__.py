"""Reference oracle for the mapped structured multigrid solve -- TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 CPU code (NumPy / SciPy) written from the paper
"Unstructured to structured: geometric multigrid on complex geometries via domain remapping"
(Nytko, MacLachlan, Moulton, Olson, Reisner, West, arXiv 2509.08109).  It exists only so that
tests, the smoke check and the benchmark's CPU-baseline leg can check and time the HIP
library against an independent implementation.  The product path (the C-ABI library and its
Python binding) never imports it, and it imports nothing from the product.

Modules
-------
fem       : pulled-back weak form (Sec. 2, eq. weak_computational), effective tensor D_c
            (Sec. 2.1), Q1 element matrices, stencil assembly with symmetric 5-value storage
            (Sec. 4.1, closing remark on storage).
boxmg     : BoxMG ingredients (Sec. 2.2): factor-2 coarsening, operator-induced interpolation
            (the cited Dendy 1982 method), Galerkin coarse operators P^T A P.
cycle     : four-colour Gauss-Seidel, V(1,1) cycle, stationary solve to a relative residual,
            float32 cycles inside float64 iterative refinement.
adjoint   : gradient of J(u) = 1/2 ||u - u_t||^2 with respect to per-cell K and the RHS.
transfer  : L2-projection transfers between a P1 mesh and the grid (Sec. 2.3): M_p, the coupled
            mass C (rasterised overlap, Sec. 2.3.1), two-iteration CG, P = M_p^{-1} C, R = P^T.

Pins (checks against facts fixed independently of this code) live in tests/test_oracle_*.py.
Parity pinned for every function here except where a docstring says "parity unpinned".
"""
