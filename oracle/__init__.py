"""CPU oracle for the Kaczmarz++ / CD++ block step (arXiv 2501.11673).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow FP64 restatement of
the paper's algorithms, used to check the GPU library.  Only the tests, the
graft smoke check and the benchmark's CPU-baseline leg may import it; the
library (``paper_2501_11673_amd``) never does, and the two share no code.  The
seeded input generators in ``synth`` are the only module both sides use.

Contents
  schedule : block schedule (SplitMix64 draws; Section 5.2, Algorithms 1, 2, 5)
  kpp      : block residual, regularized Gram, Cholesky projection, momentum
             update, adaptive rho, the solver loop, FP64 iterative refinement
  rht      : randomized Hadamard preprocessing (Definition d:rht; FHT,
             Algorithm 4; SymFHT, Algorithm 3) and the solvers with it
  lsqr     : the sketch-preconditioned LSQR projection of Kaczmarz++
             (Section 4.1; Proj of Algorithm 5)
"""
from . import schedule, kpp, rht, lsqr  # noqa: F401
from .kpp import Params, Result, solve  # noqa: F401
from .schedule import Schedule, SplitMix64, make_schedule, online_rate  # noqa: F401
