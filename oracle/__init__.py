"""FP64 CPU oracle for the gamma index (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use this
package.  The GPU library neither imports nor links it, and it imports nothing from the
GPU library.

* :func:`gamma` - Algorithm A1 of Sec. 2.1 (sorted cell table, early break, Ju's
  point-to-simplex recursion), in plain C with OpenMP over reference nodes.
* :mod:`oracle.bruteforce` - an independent exhaustive check (every face of every
  simplex, no pruning, Householder QR) for tiny grids.
"""
from .core import OracleResult, gamma, gamma_grids, simplex_dist, build, max_threads  # noqa: F401
