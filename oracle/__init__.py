"""Plain FP64 CPU oracle for the fractional control equation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library: it builds its own finite-difference matrices, calls LAPACK (through
SciPy) for the 1D eigenpairs, and solves

    (beta A^-alpha + (gamma/beta) A^alpha) u = y            (control equation)

exactly, by the spectral definition of A^{+-alpha}: transform to the tensor
eigenbasis, divide by f(lambda1_i + lambda2_j + lambda3_k), transform back.

Modules
  fd      -- 1D Sturm-Liouville FD matrices and their eigenpairs (Sec. 3.2-3.3)
  solve   -- exact solution and the eigen-coordinate error evaluators (Sec. 3.1)
  tensor  -- canonical/Tucker format definitions: full-grid evaluation, scalar
             and Hadamard products, HOSVD truncation (Appendix 1)
  brute   -- dense n^3 x n^3 brute force and the alpha = 1 sparse identity,
             used only to pin the other modules at tiny n
"""
