"""Plain FP64 CPU oracle for the P-GVIMP hot path (test infrastructure).

This package is test infrastructure only.  It is imported by the tests, by
the smoke check and by the benchmark's CPU-baseline leg, never by the
product path.  It shares no code with the HIP library: every function here
is written directly from the paper (arXiv 2411.03416, "Efficient Iterative
Proximal Variational Inference Motion Planning") in plain numpy/scipy, with
no blocking, fusion or reordering beyond what the cited passage states.

Modules and the passages they follow:
  gh         Sec. 4.3 steps 1-3 (sigma points, weights, eq. GH_quadrature_matmul)
  prior      Sec. 2.2 eq. dynamics_linear, Alg. 1 (prior kernel, Grammian, K^-1)
  gbp        Sec. 5.1 eqs. zero_mean_Gaussian, messages, belief_lambda
  sdf        grid interpolation of the signed-distance field (paper silent)
  fk         synthetic serial-chain forward kinematics (paper gives no model)
  collision  Sec. 4.1 eq. gradients_psid, eq. collision_factorization,
             eq. mapping_from_joint_to_factor, Sec. 4.3
  prox       Theorem 1 eq. mu_Sigma_update, Alg. 1, App. C step-size rule
  slr        Sec. 6.2 eqs. SLR_objective, SLR_best_ai, SLR_best_Ai, Alg. 2

Parity status: every function is pinned by the -m "not gpu" tests against
closed forms, invariants, brute force or (the hinge-cost expectation at a
converged rule, p = 30) Monte Carlo, except the hinge-cost expectation at
the small rules the workloads use, which is "parity unpinned" against the
exact integral (Gauss-Hermite is an approximation for the non-smooth hinge);
only the GPU-vs-oracle agreement at the same rule is checked there.
"""
from . import gh, prior, gbp, sdf, fk, collision, prox, slr  # noqa: F401
