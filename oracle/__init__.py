"""CPU oracle for the channel pressure-Poisson and wall-normal Helmholtz solves.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or run
this package: only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark use it. It shares no code with the HIP library.

It is plain numpy, in float64 (or np.longdouble, to measure the float64
floor), slow and direct:

* ``grid``       -- z metrics, the second-order z operator for each boundary
                    family, modified wavenumbers in the packed slot order.
* ``transforms`` -- packed real Fourier transform of the paper's App. A
                    layout, on top of numpy's FFT (a library primitive); the
                    cosine and sine transforms for walls in x or y and the
                    type-I sine transform of a field on the y faces, from
                    their definitions.
* ``tridiag``    -- subtraction-free Thomas elimination, the paper's
                    Algorithm 1 and Algorithm 2 (plain and subtraction-free),
                    the reduced boundary system of the partition method.
* ``poisson``    -- the Fourier-x, Fourier-y, tridiagonal-z Poisson solve of
                    eq. (fijk_eq) with the pinned singular zero mode, the
                    7-point residual (y periodic, or zero-gradient y walls
                    with the cosine transform), and the z-implicit Helmholtz solve of
                    eq. (proj3_impl1d).
* ``dense``      -- brute-force assembled operators for tiny grids, built
                    from face fluxes rather than from ``grid``.
* ``projection`` -- the pressure projection of a Runge-Kutta substep on the
                    staggered grid: divergence right-hand side, face
                    gradient correction, pressure update.

Every function is pinned by tests under ``tests/`` (dense brute force,
closed-form discrete eigenfunctions, direct DFT, long-double floor,
algorithm equalities); none is marked "parity unpinned" except the tanh
stretching convention, which the paper does not define.
"""
from . import grid, transforms, tridiag, poisson, dense, projection  # noqa: F401
