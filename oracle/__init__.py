"""CPU oracle for the parity-blocked rotated staggered Bloch eigenproblem.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, fp64/complex128
implementation written directly from the paper's definitions.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it;
the GPU library never does, and the GPU path shares no code with it.

Modules
-------
discretization  literal Kronecker assembly of K_l, H_l, S_d, D_d, D~_s, B_h, C_h,
                M_h and A_h (Sec. 3.1-3.3, Eqs. 3.4-3.15)
pointwise       an independent index-formula construction of the same operator
                (Bloch extension of Eq. 3.2), used for large grids and sampled
                outputs
blocks          parity classes, the block node order and Q_sigma (Sec. 4,
                Theorem 4.1, Corollary 4.2)
eigen           dense generalized eigenvalues, Gamma-point null space and the
                merged block spectrum (Sec. 4, Sec. 6, Appendix C)
fourier         Bloch Fourier bases T, F_sigma, T_sigma, symbols and the
                FFT-diagonal preconditioner (Sec. 5, Appendix B)
solve           direct solution of the shifted system (Eq. 6.2)
gradient        Hellmann-Feynman derivatives of eigenvalues with respect to the
                nodewise stiffness and density (first-order perturbation of the
                pencil of Eq. 3.15)
continuum       textbook Christoffel equation, used only as a pin

Parity status: every function is pinned by tests under ``tests/`` against
properties the paper or the mathematics fixes (see each module's header).  The
preconditioner operator K(m) = Bhat(m) C_ref Bhat(m)^H + delta*rho_ref*I is a
reading of Sec. 5.4/6.1 (the paper does not write it out); it is pinned by
being the exact inverse of A + delta*M for homogeneous material.
"""
