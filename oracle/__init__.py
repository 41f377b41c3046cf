"""CPU oracle for the recycling Krylov solvers (test infrastructure only).

This package is the plain, slow, FP64 reference that the GPU library is
checked against.  It is *test infrastructure*: only the test-suite, the smoke
entry point and the CPU-baseline leg of the benchmark may import it; the
library itself never does, and it shares no code with the library (both only
consume the seeded inputs of the separate ``workloads`` module).

Modules
  stencil  -- y = A u for 7-band structured-grid storage (Sec. 2.1, "Data
              Layout").
  precond  -- point Jacobi and the two-level Schwarz-Jacobi preconditioner
              (Sec. 2.1, "Preconditioners in GenIDLEST").
  krylov   -- GMRES(m) (Alg. 1), BiCGStab (Alg. 2), rGCROT(m,k)/GCRODR(m,k)
              (Alg. 3) with the harmonic-Ritz recycle-space update, the
              thin-QR recycle setup (Alg. 3), rBiCGStab with one
              recycle space (Alg. 4) and the hybrid rGCROT -> rBiCGStab
              driver (Sec. 2.4).

Every solver works right-preconditioned on A~ = A M^-1 in "y-space": the
iterate y approximates A~^-1 b and x = M^-1 y.

Parity unpinned: the Schwarz-Jacobi constants (subdomain size, overlap,
relaxation factors) are not given in the paper; the oracle follows the stated
reading, and its pins check it as a linear operator (brute-force dense
construction, exact-solve limit), not against the paper's values.
"""
from . import stencil, precond, krylov  # noqa: F401
