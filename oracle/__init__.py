"""CPU oracle for the 2-D five-point Jacobi sweep (test infrastructure).

This package is test infrastructure. Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import, call, link or run anything in it.
The GPU library never uses it, and it uses nothing from the GPU library.

* ``oracle.jacobi``  plain NumPy FP64 (and NumPy-float32) definitions: the sweep,
  the iterated ping-pong solver, its transpose (adjoint), the derivative with
  respect to the coefficient, the hi/lo encoding and the error bounds.
* ``oracle.cref``    a plain C + OpenMP twin of the forward solver, used to time
  the oracle on all host cores; it is bit-identical to the NumPy form.
"""

from .jacobi import *  # noqa: F401,F403
