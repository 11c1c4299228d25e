"""TEST INFRASTRUCTURE -- the oracle of the cascaded FP64x2 GEMM.

* ``ref.dd_gemm_ref``: plain FP64x2 triple-loop GEMM in C (the accuracy
  reference of Sec. 5.2); also timed as the CPU baseline.
* ``cascade``: the cascade itself (Sec. 3.2-3.4, 3.6, Appendix A) in numpy,
  step by step, for bit-level checks of the split and the exact bins.
* ``slices``: the narrow-slice (BF16/FP16/INT8) variant written out the same way.
* ``cascade3``: the FP64x3 cascade (six digits, triple-word results).
* ``illcond``: the ill-conditioned generator of the accuracy study.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path never does.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against exact rational arithmetic, closed forms, invariants or the paper's
worked example.  What no pin can fix is listed as "parity unpinned" where it
occurs: the rounding of the cascade's bin 3-6 sum (its order is free; only a
bound holds), and the FP64x3 device's triple-word summation, which is held
to the exact rounding of ``cascade3.td_round`` within a bound.
"""
