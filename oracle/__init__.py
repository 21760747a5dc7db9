"""Plain FP64 CPU oracle for the WP-CCC propagation hot path (arXiv:2403.04252).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library.

Every function follows the paper's statement of the method in plain numpy
(float64 / complex128), one step at a time, with library primitives (matmul,
LAPACK's ZGESV through ``numpy.linalg.solve``, Gauss quadrature nodes) used
only as single steps.  Where the paper is silent the module docstrings state
the reading that is taken.

Modules
-------
radial      r-grid, Simpson weights, hydrogenic bound states, Coulomb
            functions, wave-packet bins, Gram-Schmidt, the full basis
angular     Clebsch-Gordan, associated Legendre, Wigner d, Bessel J
direct      Eq. D2 radial multipole integrals and Eq. D1 direct couplings
twocentre   Eq. K1/K2 overlaps and the transfer couplings (two-centre)
propagate   Algorithm 1 (RK4 along the z-grid) for 1C and 2C
"""
