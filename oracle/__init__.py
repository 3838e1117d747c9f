"""Plain FP64 CPU oracle for the hybrid Schwarz / p-multigrid SEM solver
(Stiller, "Nonuniformly weighted Schwarz smoothers for spectral element
multigrid", arXiv 1512.02390).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library shares no code with
it: the two meet only through the seeded input generators in
``paper_1512_02390_amd.workloads``.

Everything here is written from the paper's definitions, in its order and
notation, with numpy used only for plain linear algebra (products, dense
solves).  Local subdomain problems are solved with a dense factorisation of the
restricted matrix, which is the definition the fast diagonalisation reaches
exactly; the fast-diagonalisation formula itself lives in ``schwarz.fdm_solve``
and is pinned against the dense route by the tests.

Modules
  gll             GLL points/weights, Lagrange derivative and interpolation.
  discretization  1-D assembly, the tensor-product operator, B(nu), RHS.
  weights         shape functions (Table 1), weight function, counting matrix.
  schwarz         subdomains, local solves, weighted additive Schwarz.
  multigrid       p-levels, transfers, coarse solve, V-cycle (Algorithm 3).
  mgcg            inexact multigrid-preconditioned CG (Algorithm 4).
  metrics         average logarithmic rate, n_10, cost measure.
  mlp             FP64 reference of the 2-layer weight-predictor network.
"""
