"""MI355X-native evaluation of Galerkin boundary-element weak-form entries
(3D Laplace/Helmholtz single- and double-layer, P0/P1 on flat triangles,
regular Gauss quadrature) for the rows and columns that adaptive cross
approximation requests while it fills the admissible blocks of an H-matrix.

The compute path is the C-ABI library ``libbem.so`` (HIP kernels for gfx950
plus the host-side request server, ACA and trees); ``paper_1711_01897_amd.bem``
is its thin ctypes binding.  Importing this package does not load the
library; ``inputs`` holds the seeded mesh and request generators.
"""
__all__ = ["bem", "inputs"]
