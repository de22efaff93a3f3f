"""MI355X (gfx950) dynamic optimal transport with mixed boundary conditions.

The solver is the PDHG iteration of Fitschen, Laus and Steidl for
Benamou-Brenier transport of RGB images (periodic colour axis), implemented
as HIP kernels behind the C ABI of include/ot_dyn.h; ``otdyn`` is its
Python binding.
"""
from . import otdyn  # noqa: F401
