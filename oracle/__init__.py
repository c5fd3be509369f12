"""FP64 CPU oracle for ATRG and triad-ATRG on the Ising model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP path.

The oracle is a plain, slow, readable transcription of the method of
Sugimoto & Sasaki, "Triad representation for the anisotropic tensor
renormalization group in four dimensions" (arXiv:2507.21909):

* ``linalg``  -- Householder QR (LAPACK, as a library primitive), the
  oracle's own cyclic Jacobi eigensolver and one-sided Jacobi SVD, the
  truncation rule and the sign convention.
* ``philox``  -- Philox4x32-10 (Salmon et al., SC'11) and the Gaussian
  sketch drawn from it.
* ``ising``   -- the Ising initial tensor in CP form (Sec. III), exact
  enumeration, series expansions and Onsager's solution (the pins).
* ``trg``     -- the RG step: re-split (Fig. 5f), bond swap with exact SVD or
  the randomized SVD of App. A, ATRG squeezers and coarse-graining
  (Sec. II A, makeG/makeH), the triad representation and makeMG/makeMH
  (Sec. II B), and the free energy (eq. Z).
"""
