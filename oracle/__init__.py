"""FP64 CPU oracle for the two-pass DTW nearest-neighbour search.

TEST INFRASTRUCTURE ONLY.  This package exists so that tests, the smoke check
and the benchmark's CPU-baseline leg can compare the device path with a plain,
slow, obviously correct implementation of what the paper defines.  The product
path never imports, links or executes anything in this directory, and nothing
here imports the product package.

* ``reference``  -- NumPy/pure-Python functions following the paper's definitions.
* ``native``     -- ctypes loader for ``oracle.c`` (plain C, fp64, OpenMP over
  candidates), the same definitions in a faster form for large brute-force checks.

Parity status: every function is pinned by the ``-m "not gpu"`` tests against
values the paper prints, closed forms, invariants, library special cases or
brute-force path enumeration.  The per-pass pruning counts of the parallel
search have no value printed in the paper (its figures are missing): they are
checked only through invariants relative to the exact final threshold.
"""
