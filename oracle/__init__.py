"""FP64 CPU oracle of the RIFT2 hot path (test infrastructure only).

This package is the correctness reference for the GPU library.  It is plain,
slow and written to be checked against the paper by eye:

* filterbank -- log-Gabor bank, orientation amplitude sums, maximum index map,
  noise threshold, phase congruency and its moments (Section 2.1, Feature
  Detection; Section 2.2, Feature Description);
* detect     -- FAST segment test on the normalised moment map, 3x3
  non-maximum suppression, patch-border mask, top-K (Section 2.1; Table 1);
* describe   -- dominant-index recoding (Section 3, Eqs. 1-2) and the
  6x6-cell x N_o-bin histogram descriptor (Section 2.2);
* match      -- brute-force nearest-neighbour matching (Section 4) with a
  second-neighbour ratio test;
* outliers   -- RANSAC over a similarity model (the RANSAC-like filter of
  Fig. 1's workflow) and the ground-truth metrics of Section 4.

It shares no code with the HIP path and must only be imported by tests,
the smoke check and the benchmark's CPU-baseline leg.  Functions whose result
has no independent pin say "parity unpinned" in their docstring.
"""
from .params import PCParams, DetectParams, DescParams, MatchParams  # noqa: F401
from . import filterbank, detect, describe, match, outliers, pipeline  # noqa: F401
