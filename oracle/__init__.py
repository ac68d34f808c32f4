"""Plain FP64 CPU oracle for the Newton step of the fully-coupled DG/CZM +
skeleton-lubrication hydraulic-fracture method (Giovanardi, Serebrinsky,
Radovitzky, arXiv 1911.10275).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the
package entry point and the CPU-baseline leg of the benchmark may import
this package.  The HIP library never calls it and shares no code with it.

Modules
-------
quadrature  conical-product Gauss rules on simplices
shapes      P1/P2 Lagrange bases in barycentric coordinates
mesh        topology, geometry, interface elements, skeleton pressure nodes
assemble    residual R and consistent Jacobian J = [[A, B], [C, D]]
solve       dense LU, block-Jacobi, right-preconditioned GMRES(m), GMRES-IR
newton      Newton-Raphson step and given-length load-step driver
nondim      nondimensional toughness/viscosity and closed-form LEFM checks

Parity status: every function is pinned by a CPU test (see tests/) except
where its docstring says "parity unpinned".
"""
