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
closed form, an invariant, a brute-force dense computation or a LAPACK routine.
The clover term of a random field, for which the paper prints no worked
example, is pinned by its parts: a closed form for a position-dependent abelian
flux (where each leaf sits), one for constant non-commuting SU(2) links (the
order and adjoints of the link products, which an abelian field cannot see),
and gauge covariance on random fields.
"""
from . import geometry, dirac, solvers  # noqa: F401
