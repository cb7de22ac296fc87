"""FP64 CPU oracle for the unbalanced Beckmann OT proximal iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the HIP path; the only thing both sides use is the
seeded input generator module, which holds none of the method's arithmetic.

Contents
  ops         discrete divergence D, its adjoint D*, the l2,1 / l1,1 flux
              norms, the group and scalar shrink maps, closed-form lambda_max
  sparse_ops  the same D assembled entry by entry into a sparse matrix
              (an independent second implementation used by the pins)
  uot         the primal-dual iteration (Algorithm 1) in every mode, the
              relative residual and the certified duality gap
  lp          linear-programming pins (scipy HiGHS)
  dr          an independent Douglas-Rachford solver with a dense projection
  poisson     DCT-diagonalised Neumann-Poisson solve and a direct solve
  nn          FP64 conv net forward/backward and Adam for the warm start
  admm        the ADMM solvers of Sec. IV that call the prox (Algorithm 2)

Grid convention: an image is an array of shape (ny, nx); element [j, i] is
pixel (i, j) of the paper, x fastest.  The flux M = (Mx, My) uses the same
layout; Mx[j, i] carries mass from pixel (i, j) to (i+1, j), My[j, i] from
(i, j) to (i, j+1).

Parity status: every function here is pinned by a test in
tests/test_oracle_*.py except where its header says "parity unpinned".
"""
