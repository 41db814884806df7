"""FP64 CPU oracle for the Estrada-Benzi total-communicability pipeline.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import or run anything in this package; the product path never does. It shares no code with the
HIP library (no kernels, headers, helpers, tables or constants) and imports nothing from it.

What it computes (Fioriti & Chinnici, arXiv 1409.5000, "Identification algorithm"):
  * eq. (4)  total communicability  EBTC = exp(A) 1, the row sums of the matrix exponential;
  * eq. (3)  subgraph centrality    SC = diag(exp(A))  (reference only);
  * eq. (5)  the plain sum of EBTC over the N background realizations (no averaging);
  * the K largest summed scores as the candidate target nodes ("The total communicability";
    "Multiple backgrounds scenario").
The Krylov approximation the paper relies on (the text after eq. (4), citing Afanasjew et al. 2008)
is taken as a symmetric Lanczos process; `lanczos` follows it step by step in FP64 with classical
Gram-Schmidt applied twice.

Modules
  dense     -- exp(A) 1 by eigendecomposition and by Pade expm (the plain definition, small n)
  taylor    -- exact rational Taylor series of exp(A) 1 on tiny graphs (brute force)
  tridiag   -- the small m x m exponential exp(T - theta* I) e1 of the Krylov method
  lanczos   -- the reference Lanczos approximation (same m / stop rule / shift as the HIP path)
  scores    -- realization sum (eq. 5) with a per-graph log-scale, and the top-K rule
  gradient  -- edge-weight gradient of <g, exp(A) 1> by three independent routes plus differences

Parity pins: every function is pinned by tests against closed forms, brute force, library routines
or invariants; none is marked "parity unpinned".
"""
from . import dense, taylor, tridiag, lanczos, scores, gradient  # noqa: F401

FLAG_BREAKDOWN = 1
FLAG_CAPPED = 2
FLAG_NONFINITE = 4
