"""Plain FP64 CPU oracle of the element-level finite-element hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
product path (the HIP library and its Python binding) never does, and this
package imports nothing from the product.

What it computes follows the paper's problem statement: a nonlinear residual
R(u) = 0 assembled from element contributions and its Jacobian K = dR/du
(Sec. II-A), element Jacobians gathered into a global sparse matrix by sorting
(row, col) pairs and combining duplicates (Sec. III-B), the matrix-explicit and
matrix-free operators (Sec. III-A), a Jacobi-preconditioned conjugate-gradient
solve in double precision (Sec. V-B, Fig. 4) inside Newton's method (Sec. II-A),
for a two-phase heterogeneous RVE (Sec. V-A).  Where the paper is silent
(element type, quadrature, constitutive laws, boundary treatment) the modules
state the textbook definition they follow.

Everything is float64 and written for clarity, not speed: loops over the 8
quadrature points with numpy operations batched over elements, and library
primitives (sort, dense solve) only as whole steps.

Parity status per module (what pins each one is in tests/test_oracle_*.py):
  mesh, hex8, elasticity, element, assembly, solver, j2, neohooke, adjoint, mlp:
  pinned (closed forms, invariants, brute force, finite differences).
"""
