"""FP64 CPU oracle for the matrix-free unfitted DG (SIPG) Poisson operator of
Bergbauer, Munch, Wall and Kronbichler, "High-performance matrix-free unfitted
finite element operator evaluation" (arXiv 2404.07911).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the package
entry point and the CPU-baseline leg of the benchmark may import or run this
package.  The product path (the HIP library and its Python binding) never
imports it and shares no code with it.

The oracle is deliberately plain: every quadrature point is evaluated with the
full tensor-product basis (the naive evaluation of Section 3.2), in float64,
with no sum factorisation, no blocking and no fusion.

Modules
-------
basis       Gauss / Gauss-Lobatto rules and 1D Lagrange polynomials.
geometry    Level set of a union of balls; cell and face classification.
quadrature  Dimension-reduction quadrature (Saye 2015) for cut cells, cut
            faces and the embedded interface.
operator    The bilinear form (Section 2.1 and 2.2), its action v = A u, the
            per-quadrature-point derivative with respect to the coefficient,
            term masks and an assembled sparse matrix.
solve       CG and mixed-precision defect correction drivers.
"""
