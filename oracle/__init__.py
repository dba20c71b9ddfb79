"""Plain FP64 CPU oracle of the exponential wave-propagation method.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only the tests, the smoke check and the CPU-baseline leg of the bench call it.
It shares no code, table or constant generator with the HIP library; both
sides see only the seeded inputs of the `synthetic` package.

Every function follows the paper (Ravelo, Schreiber, Peixoto, "High-order
exponential integration for seismic wave modeling", arXiv 2401.16322) step by
step in float64, with the readings of the paper's silent or garbled points
listed in the design notes. Modules:

- `operator`  : grid, damping profiles, staggered differences, H, energy (Sec. 2, Eq. 1-3, Sec. 3 Eq. 4)
- `spectrum`  : spectrum rectangle, Faber ellipse and coefficients (Sec. 3.2, Faber approximation)
- `source`    : Ricker wavelet, its derivatives, the augmented matrix tail (Sec. 3.2, Eq. 5)
- `steppers`  : Faber, Krylov (Arnoldi + Pade), RK4, RK3-2, HORK, leap-frog steps and runs (Sec. 3)
- `exact`     : the plain definitions used as pins: variation of constants by
                expm / expm_multiply with Gauss-Legendre quadrature, and the
                periodic plane-wave closed form
"""
from . import operator, spectrum, source, steppers, exact  # noqa: F401
