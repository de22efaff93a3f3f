"""Plain FP64 CPU oracle for the dynamic optimal transport solver.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code, tables or helpers with the HIP path.

Every function follows the paper (Fitschen, Laus, Steidl, "Dynamic Optimal
Transport with Mixed Boundary Conditions for Color Image Processing") and
names the passage it implements:

* ``grid``      -- the staggered discretisation of Sec. 2 (the discrete model,
                   the averaging/difference operators and boundary vectors).
* ``literal``   -- the printed matrices S_n,per, S_p, D_n,per, D_p and their
                   Kronecker assembly, for tiny grids (Sec. 2, Sec. 3).
* ``poisson``   -- the pseudo-inverse of A A^T by FFT and DCT (Sec. 3, Step 1,
                   Remark 2).
* ``prox``      -- the pointwise proximal map of J (Sec. 3, Step 2).
* ``pdhg``      -- Algorithm 1 and the reported residuals.
* ``direct``    -- a direct convex minimiser of the discrete model on tiny
                   grids (pin for the fixed point of Algorithm 1).
* ``transport1d`` -- the 1D closed form of quadratic transport through
                   quantile functions (pin for the discrete model).

All arithmetic is float64.
"""

from . import grid, literal, poisson, prox, pdhg, direct, transport1d  # noqa: F401
