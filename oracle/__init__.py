"""CPU FP64 oracle for the Frequent Directions family.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the package smoke test
and the benchmark's CPU-baseline leg use it.  It shares no code with the GPU
path; both sides meet only at the seeded input generators.

Modules
-------
fd        -- the streaming sketch (Algorithm 1 with the ReduceRank rules of
             Sections 2.3 and 3.1, SpaceSaving and Compensative FD included),
             computed through LAPACK's SVD of the buffer;
             an independent covariance-form re-derivation; a frequent-items
             counter simulation for rows that are scaled basis vectors.
evaluate  -- the error measures of Section 1.1 (covariance and projection error).
rsketch   -- the hashing and sampling sketches the paper compares against
             (Section 2.2 Hashing and OSNAP, Section 3.2 Priority and VarOpt
             sampling), with the counter-based generator they draw from.
"""
from .fd import (FD, ISVD, ALPHA, FAST_ALPHA, SSD, CFD, VARIANTS, ALL_VARIANTS, rule_indices, alpha_eff,
                 reduce_rank, SketchOracle, fd_sketch, fd_covariance_form,
                 counter_simulation)
from .evaluate import cov_err, proj_err, proj_full, tail_mass, fro2, gram, cov_err_gram

__all__ = [
    "FD", "ISVD", "ALPHA", "FAST_ALPHA", "SSD", "CFD", "VARIANTS", "ALL_VARIANTS", "rule_indices",
    "alpha_eff",
    "reduce_rank", "SketchOracle", "fd_sketch", "fd_covariance_form",
    "counter_simulation", "cov_err", "proj_err", "proj_full", "tail_mass", "fro2", "gram",
    "cov_err_gram",
]
