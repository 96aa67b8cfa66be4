"""The "dec" ordering of Sec. 5.2 / Algorithm 4 step 4.

Rows are ordered by strictly decreasing leverage score; equal scores keep
ascending row index (a stable sort), which is the reading used for ties.
"""
from __future__ import annotations

import numpy as np


def dec_order(scores) -> np.ndarray:
    """Permutation p with scores[p[0]] the largest; ties by ascending index."""
    s = np.asarray(scores)
    idx = list(range(s.shape[0]))
    # plain stable sort on the key (-score); Python's sort is stable
    idx.sort(key=lambda i: -float(s[i]))
    return np.asarray(idx, dtype=np.int64)
