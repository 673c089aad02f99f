"""FP64 CPU oracle for the reduced-KKT interior-point hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It is a plain, slow, direct implementation of what
the paper's method computes, written from the paper's definitions
(problem statement, KKT system, condensation and reduction propositions) and
sharing no code with the GPU path.  It reads its inputs from ``synthgrid``.

Modules:
  model  -- polar AC-OPF formulation in the reduced-space variable split:
            f, g, h, their Jacobians and the Hessian of the Lagrangian, from
            complex-matrix calculus (sparse scipy);
  kkt    -- IPM diagonals and residuals, and three ways to compute the Newton
            step: dense augmented system, condensed system, reduced (Schur)
            system; the reduced Hessian itself;
  ipm    -- the outer interior-point loop (filter line search, barrier
            update, inertia correction).
"""
