"""TEST INFRASTRUCTURE -- the oracle of the cascaded FP64x2 GEMM.

* ``ref.dd_gemm_ref``: plain FP64x2 triple-loop GEMM in C (the accuracy
  reference of Sec. 5.2); also timed as the CPU baseline.
* ``cascade``: the cascade itself (Sec. 3.2-3.4, 3.6, Appendix A) in numpy,
  step by step, for bit-level checks of the split and the exact bins.
* ``slices``: the narrow-slice (BF16/FP16) variant written out the same way.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path never does.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against exact rational arithmetic, closed forms, invariants or the paper's
worked example; none is "parity unpinned".
"""
