"""CPU FP64 oracle for the butterfly manifold harmonic transform (test infrastructure).

This package is test infrastructure, not product code.  Only the test suite,
the package smoke check and the benchmark's CPU-baseline leg may import it.
It shares no code with the GPU path: every function here is written from the
paper's definitions, in plain NumPy, with no blocking, fusion or reordering
beyond what those definitions state.

Modules
  modes      real Fourier modes on the flat periodic square (Sec. 1, eq. 2D-DFT;
             Sec. 5 rank analysis, eigenpairs of the periodic Laplacian)
  dense      O1: the dense transform f = Phi c and its adjoint (Sec. 1, eq.
             MHT-sum and the adjoint map to coefficients)
  butterfly  O2: the row-wise butterfly apply of a stored factor set (Sec. 2,
             block recursion and Alg. "Butterfly factorization" return set)
  sparse     the same factor set multiplied out as a product of block-sparse
             matrices (Sec. 2, Remark on the sparse-factor view); an independent
             formulation used to pin O2 at tiny sizes
  lsqr       LSQR (Paige and Saunders), the least-squares solver the inverse
             transform uses (Sec. 7.1, eq. inverse-MHT)
  interp     column interpolative decomposition of one block by column-pivoted
             QR (Sec. 2, the low-rank factorization each block takes)
  factorize  the butterfly factorization of a dense Phi with column IDs (Sec. 2,
             Alg. "Butterfly factorization"; Sec. 4 streaming order noted)
  fem        element-by-element linear finite-element stiffness and lumped mass
             on a triangle mesh, a second formulation of the cotangent Laplacian

Parity status: every function is pinned by a CPU test (tests/test_oracle_*.py).
"""
