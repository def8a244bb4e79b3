"""Plain FP64 CPU oracle of the SFC two-level overlapping Schwarz solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the
package entry file and the CPU-baseline leg of the benchmark may import it.
The product library never imports, links or executes anything here, and the
oracle shares no code with the HIP path (only the seeded input generator in
`seeded_inputs`, which holds none of the method's arithmetic).

Everything is written for a reader holding the paper (Griebel, Schweitzer,
Troska, "A dimension-oblivious domain decomposition method based on
space-filling curves"): each function cites the passage it follows.  It is
deliberately slow and plain: scipy.sparse for the matrix, Python sets/numpy
for index sets, argsort for the curve order, LAPACK Cholesky for the local
and coarse solves, textbook PCG / Richardson.

Modules
  grid       model problem and FD matrix (Sec. 3.3, eq. dof; Sec. 4)
  sfc        Z-order (Morton) curve order (Sec. 3.2, 3.3; Alg. 1 step 3)
  partition  disjoint pieces, overlap, weights, coarse blocks
             (eqs. sloc, enlarge, Di, omegai, restr)
  schwarz    local/coarse operators and the preconditioners
             (eqs. AS2a, csm, w1levprec, addSW, balan, balSW; Alg. 2)
  solvers    PCG, flexible PCG, damped Richardson (Alg. 3, eq. redrate)
  exact      DST-I diagonalisation: the exact A^{-1} f
  grad       adjoint gradient of J = 1/2 ||u||^2 w.r.t. f and a_j
"""
