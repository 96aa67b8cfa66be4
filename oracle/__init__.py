"""CPU FP64 oracle for sketched leverage scores (Chin & Liang, ACML 2018).

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
GPU library is checked against. Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library itself never
does, and shares no code, table or constant generator with it.

Contents (each function cites the passage of the paper it follows):

* ``streams``  -- the seeded random streams both sides implement from their
  published definitions: a degree-3 Carter-Wegman polynomial hash mod 2^61-1
  for the CountSketch bucket and sign (the paper only says "a pair of hash
  functions", Sec. 3.1.2), SplitMix64 for coefficient derivation, and
  Philox4x32-10 + Box-Muller for Gaussian entries.
* ``sketch``   -- CountSketch (dense and CSR) and the Gaussian sketch S*X,
  Sec. 2.1 and Algorithm 2 step 1; power-of-two column equilibration.
* ``leverage`` -- exact leverage (Sec. 2.2 definitions, Algorithm 1 in QR
  form), sketched leverage (Algorithms 2 and 3 in QR form, with a second
  Gaussian projection Pi_2), the refined variant, and the numerical-rank
  decision.
* ``order``    -- the "dec" ordering of Sec. 5.2 (stable descending argsort).
* ``metrics``  -- max relative score error and Kendall tau-b.

Parity status: every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (closed forms, invariants, brute force on tiny
inputs, published known-answer vectors); none is "parity unpinned".
"""
from . import streams, sketch, leverage, order, metrics  # noqa: F401
