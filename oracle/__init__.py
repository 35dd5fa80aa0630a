"""Plain, slow FP64 CPU oracle for the fractional-interface domain-decomposition solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call, link
or execute anything in this folder.  Only the test suite, the smoke check of the
entry module and the ``cpu_baseline`` leg of the benchmark use it.

What it computes (everything in float64, numpy/scipy only):

* ``fem``      -- P1 meshes of the unit square/cube, element-by-element assembly of
                  the stiffness and mass matrices, the free-dof ordering with the
                  interface Gamma last, and the interface operators (A_Gamma, M_Gamma).
* ``spectral`` -- the generalized eigenproblem L_h U = M_h U Lambda, U^T M_h U = I and
                  the fractional powers L_h^s = (M_h U) Lambda^s (M_h U)^T
                  (paper, Sec. 2, eq. (gevp)); the exact Schur-complement
                  preconditioner S_Gamma = K L^{1/2} + gamma L^{-1/2} (eq. (schur_precond)).
* ``system``   -- the full operator  A = K A_Omega + gamma T^T H T  with H = L_h^{-1/2}
                  (eq. (riesz), eq. (generic), the P1 realization gamma T_h^T L_h^t T_h of
                  Sec. 3), solved three independent ways (dense, sparse LU, and in 2D
                  the separable sine-transform solver), the dense interface Schur
                  complement, the discrete harmonic extension, and reference PCG drivers.
* ``ra``       -- evaluation of any rational-approximation table (c0, c_k, p_k) of the
                  solution operator c0 M^{-1} + sum_k c_k (L_h + p_k M_h)^{-1} (eq. (RA))
                  on the exact discrete spectrum, and as dense matrices.
* ``aaa``      -- a plain AAA rational approximation (Nakatsukasa, Sete, Trefethen 2018)
                  used to pin pole counts independently of the product's own builder.
* ``cnn``      -- an FP64 numpy reference of the warm-start convolutional network with
                  hand-written backpropagation.

Parity status of each function is stated in its docstring; every function here is
pinned by a test under ``tests/`` against closed forms, invariants or brute force
(see ``tests/test_oracle_*.py``).
"""
