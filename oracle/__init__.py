"""CPU oracle for butterfly supports, bitruss numbers and the BE-Index.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the GPU path
(`paper_2001_06111_amd`) and neither imports the other.

  bt_oracle.c  plain C (OpenMP) counting and level-synchronous peeling with
               explicit butterfly enumeration, from the definitions of
               Section II of the paper.
  brute.py     brute force over vertex quadruples and the k-bitruss
               fixpoint definition, for tiny graphs; the one-edge-at-a-time
               peel of the baseline algorithm (Algorithm 1).
  index_def.py the maximal priority-obeyed blooms straight from their
               definition (Section IV, Definitions 6-8).
  query.py     connected components of a k-bitruss (Definitions 4-5) by
               breadth-first search.

Functions take a graph as (n_upper, n_lower, row_ptr, col): upper-major
CSR with int64 row pointers and int32 lower ids sorted per row; edge e is
CSR position e.
"""
from .api import support, bitruss, edge_support, lib_path, build, max_threads  # noqa: F401
