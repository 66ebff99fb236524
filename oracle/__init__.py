"""FP64 CPU oracle for the FastVEM pressure projection (test infrastructure).

This package is a plain, slow, independent restatement of the paper's method:
binary-space cut cells (Sec. 5.1), the conforming VEM of orders 1 and 2
(Sec. 3.1, App. A), the divergence right-hand side (Sec. 3.2), the nested
boundary-aware hierarchy (Sec. 5.2), the diffusion-free prolongation and
Galerkin coarse operators (Sec. 4), the Chebyshev-smoothed V-cycle and the
preconditioned CG solve (Sec. 4, Sec. 6 "Multigrid Method Evaluation").

It exists only to check the product.  Only the test suite, the smoke entry
point and the benchmark's CPU-baseline leg may import it; the product never
calls it, and it shares no code with the product.  Where the paper is silent,
the reading taken is stated at the function that takes it.

Parity unpinned (no printed value or closed form fixes them; they are
conventions that both sides must merely agree on): the triangle ordering
tie-breaks of the cut-cell construction, the tolerance choices, the
stabilisation scale h_E, the Chebyshev interval, and the hierarchy tie-breaks.
"""
