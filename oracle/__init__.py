"""Plain FP64 CPU oracle for the kernel-independent FMM (3D Laplace).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP path (no kernels,
helpers, tables or constant generators); the two are compared only through
their outputs on identical seeded inputs.

The oracle follows the paper's shared-memory FMM (Section 2.1, Algorithm 1)
with the operators of Table 1, written step by step in double precision and
single-threaded:

* ``kernel``    -- the Laplace kernel 1/|x-y| and its gradient (eq. (2)).
* ``direct``    -- the direct sum of eq. (1); the exact result the FMM
                   approximates.
* ``tree``      -- the uniform octree of Section 2.1, Morton keys, and the
                   U and V interaction lists of Table 1.
* ``surface``   -- the kiFMM check/equivalent surfaces with
                   n = 6(p-1)^2 + 2 points (Section 4, message-size formula).
* ``operators`` -- truncated-SVD pseudo-inverses and the translation
                   operators S2U, U2U, U2D, D2D of Table 1, plus the
                   SVD compression of the U2D (M2L) operators.
* ``fmm``       -- Algorithm 1 steps (1a) S2U, (1b) U2U, (2a) VLI, (2c) D2D,
                   (3b) D2T and (3c) ULI; and the derivative of the evaluate
                   for a weighted sum of the potentials (``fmm.vjp``).

Readings of points the paper leaves open (kernel normalisation, coincident
points, surface geometry, pseudo-inverse cutoff, compression scheme) are
stated in the module that implements them.

Pins: each module is checked by tests/test_oracle_*.py against something other
than itself -- closed forms, the direct sum, brute force on tiny inputs,
invariants (linearity, translation, symmetry of the derivative), convergence in
the expansion order, and the values the paper prints.  The readings above are
choices the paper does not fix; for them parity is unpinned: another valid
choice (other surface radii, cutoffs or compression bases) gives a different,
similarly accurate kiFMM.
"""

from . import kernel, direct, surface, tree, operators, fmm  # noqa: F401
