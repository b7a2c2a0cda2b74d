"""FP64 CPU oracle for Sinkhorn Word Mover's Distance (arXiv 2107.06433).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; the two meet only on the raw arrays drawn by
``paper_2107_06433_amd.synth``.

Contents
--------
``wmd``   the method written out plainly in float64: query selection
          (Algorithm 1, first step), the Euclidean cost matrix, the dense
          Sinkhorn-Knopp iteration of Algorithm 1 / Table I over the whole
          vocabulary, and the same iteration restricted to each document's
          support.
``emd``   exact earth mover's distance by linear programming and by brute-force
          vertex enumeration; used only by the tests that pin the oracle.
"""
from .wmd import (  # noqa: F401
    select_query,
    normalized_columns,
    cost_rows,
    sinkhorn_scalings,
    sinkhorn_scalings_until,
    sinkhorn_wmd_dense,
    sinkhorn_wmd_support,
    transport_plan,
    wmd_dense_corpus,
)
