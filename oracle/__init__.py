"""Plain FP64 CPU oracle for the neural-quantum-state VMC hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the bench's
CPU-baseline leg may import this package.  The library under
``paper_2108_03409_amd`` never calls into it, and this package imports nothing
from there: the two share no code, tables or constants.

Every function restates the definition from the paper (Schmitt & Reh, "jVMC:
Versatile and performant variational Monte Carlo leveraging automated
differentiation and GPU acceleration", SciPost Phys. Codebases) in float64 /
complex128 NumPy, without blocking, fusion or reordering beyond what the
definition states.  Where the paper is silent the reading taken is stated in
the function's docstring.

Modules
  lattice    bond lists and the connected configurations of the two Hamiltonians
  rbm        restricted Boltzmann machine log-amplitude and log-derivatives
  cnn        two-layer periodic CNN log-amplitude and log-derivatives
  eloc       local estimator E_loc and the exact-enumeration expectation value
  philox     Philox4x32-10 counter-based generator and its integer/uniform maps
  metropolis Metropolis chains and the exact transition matrix
  sr         quantum Fisher matrix S, force F, diagonal shift, Cholesky solve
  made       masked autoregressive proposal network (MADE) and exact MH mixing
  ess        integrated autocorrelation time and effective sample size
"""
