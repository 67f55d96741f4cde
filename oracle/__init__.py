"""Oracle: a plain, slow, obviously-correct FP64 CPU evaluation of the ADER-DG
element kernels for the linear elastic wave equation on tetrahedra (Uphoff &
Bader, "Yet Another Tensor Toolbox", Sec. 5.1, Eqs. seissol:derivative,
seissol:timeint, seissol:correction_local, seissol:correction_neigh).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import or run it.  The product path
(the HIP library and its Python binding) never imports, links or calls
anything here, and nothing here imports the product.  The two share no code:
the oracle builds its own reference matrices (exact polynomial arithmetic +
Golub-Welsch Gauss-Jacobi quadrature), its own star and flux-solver matrices
(explicit 9x9 eigen-decomposition/inverse) and evaluates every contraction as
literal loop nests over full index ranges (oracle/stages.c).

Modules
  refmat    Jacobi polynomials, Gauss-Jacobi rules, Dubiner bases, M, S, K-hat,
            K-tilde, R, R-hat, f  (Sec. 5.1.1 matrix shapes; weak form Sec. 2)
  elements  geometry, star matrices, Godunov flux-solver matrices A+/A-
  stages    ctypes binding of the C loop nests + pure-Python brute-force sums
  madness   the separable contraction of Sec. 7 (Eq. stock_mra): the paper's
            six-step chain of one-index contractions, and the literal sum
"""
