"""Reference CPU oracle for the columnar ABM hot path (TEST INFRASTRUCTURE).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library under
``paper_2601_16292_amd``; neither imports the other.

Modules:
  thresholds -- exact uint32 Bernoulli thresholds from rational beta, gamma
                (Python ``fractions.Fraction``);
  oracle     -- ctypes wrapper of the plain single-threaded C oracle
                ``amber_oracle.c`` (built to ``liboracle.so`` by ``build_oracle``);
  brute      -- pure-Python brute force for tiny populations (its own
                Philox, O(N^2) neighbour search), used to pin the C oracle.

The oracle also holds the view primitives of Sec. 3.3 (full and filtered
updates, id-indexed scatter-add on int32 / float32 columns) and resuming a
run from host columns.

Parity status: every function is pinned by the ``-m "not gpu"`` tests
(rocRAND's Philox engine, mpmath/Decimal thresholds, numpy's ``add.at`` and
int32 arithmetic, mpmath's exact fused multiply-add, SplitMix64's published
outputs, invariants on planted bad rows, brute force, closed forms).
Nothing here is "parity unpinned".
"""
