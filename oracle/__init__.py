"""FP64 CPU oracle for the QCD+QED O(a)-improved Wilson-Dirac operator.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this package.  The HIP library never
calls it, shares no code with it, and must fail loudly when its own extension
is missing rather than fall back to anything here.

The oracle is the plain definition of each quantity, written with numpy in
complex128: full 4x4 gamma products, explicit 12x12 clover matrices, LAPACK
inverses, textbook Krylov solvers.  Each function names the passage of the
paper (arXiv:2502.02490) it follows; where the paper is silent, the reading
taken is stated in the docstring.

Modules
  geometry  site indexing: eq. (lexi), eq. (ipt), parity, neighbours
  dirac     gamma matrices, U(3) links, hopping term, clover term, D, Schur D-hat,
            clover packing (Sec. 4.1.3)
  solvers   CGLS, GCR(m), FGCR(m), even-odd prepare / solve / reconstruct
  ptc       parallel-transport convolution network (forward, gradients, Adam)

Parity status: every function is pinned by a `-m "not gpu"` test against a
closed form, an invariant, a brute-force dense computation or a LAPACK routine,
except the clover values of a generic random field, which are pinned only by
invariants and by closed forms for abelian fields ("parity unpinned" beyond
those; the paper prints no worked example).
"""
from . import geometry, dirac, solvers  # noqa: F401
