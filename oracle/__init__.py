"""Reference ("oracle") implementation of the pressure-Poisson / projection path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
calls it and shares no code with it.

Everything here is plain, slow, obviously-correct FP64 arithmetic written from
the paper (Verzicco-Orlandi staggered finite differences, AFiD; Sec. 2.1-2.2):

* ``grid``      - metrics of the stretched wall-normal grid and the modified
                  wavenumbers of the periodic directions.
* ``operators`` - discrete divergence, gradient, Laplacian (flux form),
                  wall-normal second differences.
* ``poisson``   - the direct Poisson solve (2-D FFT in the periodic plane, one
                  tridiagonal solve per wavenumber pair) and the projection /
                  pressure update.
* ``cn``        - wall-normal Crank-Nicolson solves.
* ``substep``   - explicit terms, CFL number and one RK3 substep.
* ``timestep``  - the full RK3 step, the Courant-limited time step, wall-normal
                  statistics.
* ``multires``  - the multiple-resolution temperature grid (Sec. 6): velocity
                  prolongation, temperature restriction, the temperature step
                  on its own grid and the coupled step.

Library primitives used as steps: ``torch.fft.rfft2 / irfft2`` (the 2-D real
FFT), ``math.fsum`` (exactly rounded sums).  Adjoints are obtained with
``torch.autograd`` through these same functions, independently of the GPU
library's hand-written adjoints.

Parity status of every function is listed in the module that defines it; every
reading has an independent pin (the temperature update order of the substep
by the third-order time convergence of Sec. 2.1, see ``substep``).
"""
from .grid import Grid  # noqa: F401
from . import operators, poisson, cn  # noqa: F401
