"""CPU FP64 oracle for the exponential time propagator (TEST INFRASTRUCTURE).

A plain, slow, readable restatement of what the paper's method computes, used
only to check the HIP implementation.  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code with the HIP path (the two meet only at the seeded input
generators in ``workloads``).

Modules
  fem       hex8 shape functions, quadrature, lumped mass, loads, K, R(u), H(u)x
  material  strain energies, stresses and the secant split R(u) = H(u) u
  krylov    Arnoldi with modified Gram-Schmidt, exp(H_m), error estimate, expv
  stepper   first-order system, midpoint Magnus step, predictor-corrector
"""
