"""FP64 CPU oracle for the Nystrom-preconditioned matrix-free NGD hot path.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously-correct NumPy implementation of
what the GPU library computes, used to check it. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the library and its Python binding never do, and this package imports
nothing from them (it reads its inputs from `workloads`, which holds data only).

Contents, each following the passage of arXiv 2505.11638 it cites:

* `mlp`      tanh MLP ansatz (Section 2.3), forward Taylor-mode propagation of value, gradient,
             Laplacian and time derivative, residuals of the Poisson (eq. energy_poisson) and heat
             (eq. heat_energy) least-squares energies, the exact reverse-mode residual Jacobian
             (Section 4.1.1) and the gradient.
* `navier_stokes`  the steady Navier-Stokes rows of the Kovasznay flow (Section 5.1.3, eq.
             navier_residual): velocity and pressure networks, residual rows, loss and the exact
             Gauss-Newton Jacobian by the reverse sweep with per-row seeds.
* `linalg`   the Gramian G = J^T W J of Theorem thm:matfree (eq. G_matrixfree), its damped matvec,
             and the direct solve of Alg. 2 (Cholesky) with two independent cross-checks.
* `nystrom`  Alg. 6 (randomized Nystrom, stable form) taken step by step, the Nystrom approximation
             by its definition (eq. nystrom_approx), and the preconditioner of eq. nystrom_inverse.
* `cg`       preconditioned conjugate gradients as used by Alg. 3.
* `ngd`      the damping rule (Section 4.3 and the experimental setup of Section 5), the power method,
             Armijo backtracking and one step of Alg. 1 with Alg. 3 + Alg. 4 at a fixed sketch size.
* `philox`   the Philox4x32-10 counter-based generator (Salmon et al., SC'11) with Box-Muller, used to
             check the GPU's on-device Gaussian test matrix.

Every function is pinned by `tests/test_oracle_*.py` against finite differences, closed forms,
invariants and brute force, not against itself.
"""
