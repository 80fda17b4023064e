"""Plain FP64 CPU oracle for FEM harmonic inpainting with optimised data.

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously correct
reference that the GPU library is checked against. Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never does, and it shares no code with it.

Arithmetic is float64 throughout; integer work (mesh, indices) is exact.
Each module cites the passage of Chizhov and Weickert, "Efficient Data
Optimisation for Harmonic Inpainting with Finite Elements" (arXiv 2105.01586)
that it follows:

* ``quadtree`` / ``mesh``: the adaptive triangle mesh whose vertices include
  every mask pixel (Section 2.2). The paper builds a Delaunay triangulation of
  the mask pixels plus random unknown vertices; this oracle (like the GPU
  library) uses the 2:1-balanced quadtree triangulation refined to unit cells
  at every mask pixel, whose right isosceles triangles are non-obtuse and so
  themselves satisfy the Delaunay criterion.
* ``fem``: linear (P1) finite-element stiffness matrix, Dirichlet rows at mask
  vertices, reflecting boundary as the natural boundary condition (Section 2.1
  eqs. (1)-(3), Section 2.2).
* ``solve``: the harmonic extension by a direct sparse Cholesky factorisation
  (never CG), so the GPU's iterative answer is compared against an exact one.
* ``raster``: linear interpolation inside each triangle to every pixel
  (Section 2.2, last paragraph).
* ``error``: squared error map, mean squared error and per-triangle L2 error
  (Section 3).
* ``tonal``: u = B g, its adjoint, and least squares g* = argmin ||B g - f||^2
  through the normal equations B^T B g = B^T f (Section 4, eqs. (4), (5)).
* ``densify``: global top-k error-driven mask growth, and the paper's
  per-triangle densification (Section 3).
* ``colour``: the method channel by channel on one shared mesh (Section 5).
* ``delaunay``: the paper's own mesh, a Delaunay triangulation of the mask
  pixels and the unknown vertices (Section 2.2), made unique by symbolic
  perturbation where vertices are cocircular.
* ``l1``: tonal optimisation for the L1 error by iteratively reweighted least
  squares (the paper's large colour example; it states no method).
"""
