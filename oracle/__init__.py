"""CPU float64 oracle of the low-Mach variable-density RK substep.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import, call or execute anything in this
package.  It is written from the paper (Reuter, Oliver & Moser, "A
pseudospectral method for direct numerical simulation of low-Mach,
variable-density, turbulent flows") and shares no code with the HIP library:
no kernels, headers, helpers, tables or constant generators.  Library
primitives used as steps: numpy FFT, LAPACK banded LU (scipy), dense solves.

Parity status of each function is stated in its module; every function here
is pinned by a CPU test against values fixed by the paper or by mathematics
(brute-force sums, closed forms, library routines, invariants, special cases).
"""
from .bspline import SplineSpaces, basis, clamped_knots, derivative_map, greville  # noqa: F401
from .fourier import n_of_index, to_physical, to_spectral, wavenumbers  # noqa: F401
from .lmvd import (Config, Integrator, Plan, bdf_coefficients,  # noqa: F401
                   curl_free_momentum, divergence_free_momentum, substep)
