"""CPU oracle for the FFT-based Bloch-wave method (Segurado & Lebensohn).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 restatement of
what the method computes, used to check the HIP path.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never routes through it, and it imports nothing from the product package
except the seeded input generators (`paper_2106_12487_amd.inputs`), which hold
none of the method's arithmetic.

Modules
-------
fourier    own DFT (per-axis DFT matrices applied as matrix products) and the
           discrete frequencies (Sec. 3.1 eq. "frequencies", Sec. 3.2)
operators  stiffness / mass / inverse-mass operators (Sec. 3.2 eqs. hatA,
           hatM; Sec. 3.3 eq. def_invM) and the homogeneous-reference
           preconditioner (Sec. 3.3 eqs. matrixP, precond)
solvers    preconditioned CG (Algorithm "InvA"), subspace iteration (Algorithm
           "subspace"), shift-invert implicitly restarted Lanczos (Sec. 3.3),
           dense generalized eigendecomposition and the Gamma-point deflation
postproc   group velocity of the branches (Sec. 5.1 eq. c_group) and their
           long-wave speeds, with the Voigt/Reuss bracket

Every function is FP64 and works in SI units.  Parity status of each function
is listed in its docstring; none is "parity unpinned" unless it says so.
"""
