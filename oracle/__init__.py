"""FP64 CPU oracle for the finite-strain tangent apply v = K(u) w.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
package: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library (no tables, no
kernels, no helpers) and it never reads a value produced by the HIP path.

What it computes is the plain definition of the discrete tangent of the paper
(Sec. 2.1, eqs. for the weak form F, its Gateaux derivative K and the tangent
stiffness tensor L; Sec. 2.4 for the cell-wise quadrature), for the
compressible neo-Hookean energy of Sec. 3.2, written without sum
factorization, without caches and without the directional-derivative trick:
the 81-entry tangent tensor L is formed explicitly at every quadrature point
and contracted with full (p+1)^3-term basis gradients, both

* assembled into a sparse matrix (the "classical" sparse baseline, Sec. 3.2.2),
  then multiplied with w, and
* as a naive element loop that never forms a global matrix.

Modules
-------
basis     1D Gauss rule, Gauss-Lobatto-Legendre support points, Lagrange basis
mesh      Q_p box and general hexahedral meshes: numbering (the canonical
          order of the library for general meshes), trilinear geometry,
          basis gradients
material  energy, first Piola-Kirchhoff stress, explicit tangent tensor
material_split  the same for the split (isochoric-volumetric) neo-Hookean law
fem       state, residual, energy, assembled tangent, naive apply
linelast  textbook small-strain stiffness B^T D B (pin for the u = 0 limit)
solver    Newton on the weak form with assembled tangent and direct solves
net       the learned smoother's convolutional network: forward, loss,
          parameter gradients, Adam step, patch node map
csr_spmv.c  y = A x for an assembled CSR matrix on all host cores (OpenMP):
          the assembled-matrix baseline the benchmark's CPU leg times on the
          oracle's assembled tangent (compiled by build_c.py)

Every function is float64 unless it is fed complex128 input for the
complex-step pins, in which case it works in complex128 throughout.
"""

from . import basis, mesh, material, material_split, fem, linelast, solver, net  # noqa: F401
from .mesh import BoxMesh, HexMesh  # noqa: F401
