"""k-NN classification by majority vote, the classification application of the
paper's Section 2.2: a query takes the class most represented among its k
nearest references (Euclidean, FP64 brute force from ``oracle.knn``).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

Reading where the paper is silent: a tie between classes goes to the class of
the nearest neighbour among the tied classes (neighbours in (distance, index)
order).
"""
from __future__ import annotations

import numpy as np

from . import knn


def vote(neighbour_labels) -> int:
    """Majority label of one query's neighbours, given nearest first."""
    labels = [int(x) for x in neighbour_labels]
    counts = {}
    for lab in labels:
        counts[lab] = counts.get(lab, 0) + 1
    top = max(counts.values())
    for lab in labels:  # nearest first: the first label with the top count
        if counts[lab] == top:
            return lab
    raise AssertionError("unreachable")


def classify(Q, R, labels, k: int, threads: int = 0) -> np.ndarray:
    """Predicted label of every query (int64)."""
    _, idx = knn(np.ascontiguousarray(Q, dtype=np.float32), np.ascontiguousarray(R, dtype=np.float32), k, "l2",
                 threads=threads)
    labels = np.asarray(labels)
    return np.array([vote(labels[row]) for row in idx], dtype=np.int64)
