"""FP64 CPU oracle for the preconditioned GCR(k) depth solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only the tests, the entry point's smoke check and
the benchmark's CPU-baseline leg do.  It shares no code with the HIP path.

It restates, plainly and slowly, what the paper's elliptic solver computes
(Ackmann, Dueben, Palmer, Smolarkiewicz, "Mixed-precision for linear solvers
in global geophysical flows", arXiv:2103.16120):

* ``operator``  -- grid, Earth constants, the coefficient fields of the
  elliptic problem obtained from the linearised pressure gradient (eq.
  rhslin) and the pointwise 2x2 inversion (eq. Qexpr), and the discrete
  generalised Laplacian L (eqs. Elliptic, L_Operator) with the residual
  (eq. Residual); Section 2.2.
* ``precond``   -- preconditioner options 0-3, option 3 being the
  semi-implicit Richardson scheme of eq. P_Operator; Section 2.3.
* ``gcr``       -- the GCR(k) iteration with the exit condition of eq.
  exitcondition and one enforced full cycle; Section 2.3 (its flowchart,
  Fig. 1, is not available, so the step order is the one its text names:
  step 1 initial residual, step 2 update + exit test, step 3 preconditioner
  and operator, step 4 orthogonalisation).
* ``cnn``       -- plain float64 reference of the learned preconditioner's
  3x3 convolution network (forward and gradients).  Not from the paper.

Readings of places where the paper is silent are listed in each module.
"""
