"""Plain FP64 CPU oracle for the per-time-step analytical adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark can check the HIP implementation against an
obviously-correct restatement of the paper ("Fast and Reliable Gradients for
Deformables Across Frictional Contact Regimes", arXiv 2603.16478).

It shares no code with the HIP path; both take their inputs from the seeded
generators in ``synth``.  Every function cites the passage it restates.

Modules
  fem       discretisation: rest-shape operators G_i, volumes, lumped mass,
            Lame parameters, the constant system matrix A (Sec. 3.3)
  elastic   Neo-Hookean local projection and its SVD-based Jacobian
            (Sec. 5.3, App. B.0-B.4)
  fb        smoothed Fischer-Burmeister function and its partials (Sec. 5.2)
  contact   contact candidates and frames, contact-aligned rotation R,
            contact Jacobian blocks K_c and k_mu (Sec. 5.2, App. A.1)
  forward   damped Newton solve of the coupled residual (Sec. 3, eq:dynamics)
  adjoint   explicit adjoint matrix, direct sparse LU solve with refinement,
            gradient contractions (Sec. 5.1, 5.4, App. B.3)
  woodbury  dense Woodbury preconditioner for small checks (Sec. 5.4)
  rollout   multi-step rollout and backward recursion (Sec. 5.1)

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(closed forms, invariants, finite differences or brute force); see the test
files named in each function's docstring.
"""
