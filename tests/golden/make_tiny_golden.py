"""Write tiny_wmd.txt from the FP64 oracle (dense, full-vocabulary form)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2107_06433_amd import synth  # noqa: E402


def main():
    w = synth.make_workload("tiny")
    c = w.corpus
    ids, qw = w.queries.query(0)
    out = oracle.wmd_dense_corpus(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, w.lam, w.max_iter)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_wmd.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle, workload 'tiny' (seed 1001), lambda=10, 15 iterations; one value per document\n")
        for v in out:
            f.write(f"{v:.17g}\n")


if __name__ == "__main__":
    main()
