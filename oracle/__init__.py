"""FP64 CPU oracle for the particle-mesh force-and-step loop.

TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package. The product path (the
HIP library and its Python binding) never imports, calls or links it, and this
package imports nothing from the product path; the two share no code.

Contents
  pm       mass assignment, exact 7-point Poisson solve, FFT solve, 5-point
           gradient, interpolation, kick-drift-kick (paper Sects. 3.1-3.8)
  mg       FP64 multigrid V-cycle following the paper's steps (Sects. 3.6-3.7)
  adjoint  vector-Jacobian products of the above and the reverse leapfrog
  ics      Lagrangian-perturbation-theory initial conditions (1LPT to 3LPT) and the
           power-spectrum estimator (paper Sects. 3.3, 4)
  gravity  background expansion with a cosmological constant, parametrised gravity
           mu(a) and QUMOND (paper Sects. 2.3, 2.4, 3.1, 3.10)
  fr       f(R) gravity (Hu-Sawicki): the scalaron by non-linear multigrid with the
           closed-form cubic and quartic roots (paper Sects. 2.5, 3.7.2, 3.11)

Every function is plain numpy/scipy in float64, written for readability.
"""
from . import pm, mg, adjoint, ics, gravity, fr  # noqa: F401
