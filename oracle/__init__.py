"""Plain, slow, FP64 CPU oracle for the EQS explicit-RKC hot path.

TEST INFRASTRUCTURE ONLY. The oracle is imported by ``tests/``, by
``__graft_entry__.smoke()`` (to check the GPU result) and by the
``cpu_baseline`` leg of ``bench.py``. The product library never imports,
links or calls anything here, and this package imports nothing from the
product package; the two share only the seeded input generator ``eqsgen``,
which holds no arithmetic of the method.

What it computes (Richter, Schoeps, Clemens, arXiv 1612.09447):
  * ``fem``   - P1 element gradients, assembly of the permittivity matrix M
                and of frozen conductivity matrices, the product K(x)x by an
                element loop (Sec. II eq. (1)-(2), Sec. III), CSR products and
                a symmetric-Gauss-Seidel PCG used as an accurate M-solver.
  * ``rkc``   - Runge-Kutta-Chebyshev coefficients and one step (Sec. II,
                ref. [9]: Sommeijer, Shampine, Verwer 1998).
  * ``eqs``   - the semi-discrete right-hand side F(t, Y) = M^{-1}(b(t) -
                K(x)x) with Dirichlet elimination, explicit Euler (eq. (3)),
                RKC trajectories, and the stability-bound check.
  * ``guess`` - start vectors: modified Gram-Schmidt (eq. (4)), the Galerkin
                projection (eq. (5)), POD bases (Sec. IV).
  * ``mlp``   - FP64 forward/backward of the start-vector network.

Every function cites the passage it follows. Pins live in ``tests/``.
"""
