"""Plain FP64 CPU oracle of the SEIRD implicit step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product (the HIP
library and its Python binding) never imports, links or calls it, and the
oracle shares no code with the product beyond the seeded input generators
of ``seird_inputs`` (which hold none of the method's arithmetic).

Modules
-------
fem      geometry, lumped mass, reaction, residual, exact Jacobian
         (Eqs. seird1-5, N, vec_component1/2, timediscrete, weakform)
newton   fully coupled Newton time step, Picard and Picard-Gauss-Seidel
         cross-checks (Eq. weak_vec_implicit, Appendix A)
krylov   right-preconditioned restarted GMRES with PETSc-style stopping,
         one-level RAS and the multiplicative two-grid preconditioner
         (Section 3, Eqs. RAS, presmoother/coarsecorrection/postsmoother)
ode      per-node ODE limit (Appendix B.4)
mms      manufactured forcing and observed order (Appendix B.1, Eq. MMS_order)
adjoint  discrete adjoint of a case-count misfit

Pins (what each function is checked against) are listed in the test files
``tests/test_oracle_*.py``.
"""
