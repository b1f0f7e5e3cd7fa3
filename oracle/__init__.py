"""FP64 CPU oracle for the rank-structured supernodal Cholesky solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, independent
restatement of what the method computes (NumPy / SciPy LAPACK, FP64).  Only
``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg
may import or call it.  The product path (the HIP library and its Python
binding) never imports it, and it imports nothing from the product.

Parity status per function (what pins it, see the tests named ``test_oracle_*``):

* ``ordering.nested_dissection`` / ``symbolic``: valid permutation, separator
  property, union pattern contains the true Cholesky pattern, the descendant row
  property of §2.1, the scatterRows worked example of §2.1.
* ``factor.factor`` (exact): dense Cholesky of the permuted matrix (uniqueness).
* ``factor.factor`` (compressed): full-rank sampling reproduces the exact factor;
  exactly low-rank blocks are recovered; ``U^T U = I``, ``V = L^O U``; every
  pivot positive (§3.2); approximation error against the SVD bound.
* ``factor.offdiag_multiply`` / ``offdiag_multiply_transpose`` (Algorithm 2 and its
  transpose): the explicit block product ``L^O_j G`` with ``L^O_j`` formed by the
  triangular solve of Algorithm 1, with explicit and with compressed descendants;
  ``compress_implicit`` reproduces the explicit compression (ranks, ``V_j U_j^T``).
* ``diagonal`` (§4.1-4.2, §5.3: coordinate split, block tree, Algorithms 4-6): hand-worked
  splits and tree labels; Algorithm 4 against a dense triangular solve of the written-out
  tree; full-rank sampling reproduces the dense Cholesky factor; every leaf and low-rank
  block satisfies the block-Cholesky recurrences of the written-out factor (Schur
  complement, ``V_s = L(R_s, C_s) U_s``, ``U_s`` orthonormal and spanning the sample);
  the restart policy on a planted failure.
* ``solve.apply_preconditioner(interior=True)`` / ``interior_blocks`` (§5.1): the closed
  form ``L(R^B, C^B) = A(R^B, C^B) L(C^B, C^B)^{-T}`` against the block the factorization
  computes, ``L(C^B, C^B)`` against the block's own dense Cholesky factor, the blocks'
  maximality, and the apply through eq. interiorBlockMult against the stored-block apply.
* ``philox``: the published known-answer vectors of Philox4x32-10.
* ``spectral.spectral_coordinates`` (§4.3, block Lanczos on the graph Laplacian): the
  closed-form spectrum and cosine eigenvectors of grid graphs (distinct modes, and the
  threefold axis mode of a cube), a dense eigen-decomposition when the Krylov space is the
  whole space, and a hand-built Laplacian.
* ``solve``: exact factor gives ``M^{-1} = A^{-1}``; symmetry and positivity of
  the rank-structured preconditioner; manufactured solutions.
* ``adjoint``: central finite differences of dense solves.
* PCG iteration counts of the rank-structured preconditioner: parity unpinned by
  the paper (checked only against this oracle's own count).
"""
