"""CPU FP64 oracle for the embedded-boundary AMG-PCG solve.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of what the method computes, written from the paper
(Peng, Appelo, Liu, "Universal AMG accelerated embedded boundary method
without small cell stiffness").  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product library never
calls into it and it shares no code with the GPU path.

Modules
  eb_assembly  classification, line-by-line diagonal, cut records, RHS, CSR
  spd          the 1-D segment matrices and the SPD criteria of Sec. 2.4
  amg          box aggregation, smoothed prolongator, Galerkin products,
               coarsest Cholesky, V(1,1) cycle
  pcg          preconditioned conjugate gradients and direct references
  learned      the learned fine-smoother extension: network, weighted cycle,
               loss and gradients
  steppers     theta-scheme (wave) and Crank-Nicolson (heat) time steppers
  qoi          quantities of interest over a family of geometries (Sec. 3.6)

Parity status per function is stated in each module header.
"""
