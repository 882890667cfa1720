"""CPU FP64 oracle for the VMS / generalized-alpha Newton step (TEST INFRASTRUCTURE).

This package is a plain, slow, obviously-correct NumPy/SciPy implementation
of what the GPU hot path computes.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does,
and it shares no code with the HIP library (both read the seeded inputs from
``synth``).

Where the paper gives a plain definition the oracle writes that definition
out (the linear solve is Delta = -K^{-1} R by sparse LU; the tangent is the
exact derivative of the residual, obtained by complex-step differentiation
instead of the closed forms of the consistent-linearization appendix).  Where
the method is itself a procedure (generalized-alpha staging, the predictor
multi-corrector loop, the Schur-complement-reduction preconditioner, FGMRES)
the oracle follows the paper's steps in order.

Modules
  material  constitutive relations (Gibbs energy -> rho, beta; iso Piola stress)
  element   quadrature, element residuals, complex-step element tangents
  assemble  global residual/tangent, Dirichlet rows, symmetric diagonal scaling
  newton    generalized-alpha predictor multi-corrector time step
  krylov    plain GMRES / FGMRES and the exact block preconditioners
  full3     the unreduced 3-field (u-dot, p-dot, v-dot) Newton system
"""
