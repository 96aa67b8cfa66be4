"""Error metrics reported beside every result.

* max relative score error: max_i |a_i - b_i| / b_i over b_i > 0, with rows of
  zero reference score required to be exactly zero;
* Kendall tau-b between two score vectors (scipy's O(n log n) routine, pinned
  against an O(n^2) pair count in the tests).
"""
from __future__ import annotations

import numpy as np
from scipy import stats


def max_rel_err(est, ref) -> float:
    est = np.asarray(est, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    pos = ref > 0
    zero_ok = np.all(est[~pos] == 0.0)
    if not zero_ok:
        return float("inf")
    if not pos.any():
        return 0.0
    return float(np.max(np.abs(est[pos] - ref[pos]) / ref[pos]))


def kendall_tau(a, b) -> float:
    return float(stats.kendalltau(np.asarray(a, dtype=np.float64),
                                  np.asarray(b, dtype=np.float64)).statistic)


def kendall_tau_bruteforce(a, b) -> float:
    """O(n^2) tau-b, for pinning the library routine on small inputs."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = a.shape[0]
    conc = disc = ties_a = ties_b = 0
    for i in range(n):
        da = np.sign(a[i + 1:] - a[i])
        db = np.sign(b[i + 1:] - b[i])
        prod = da * db
        conc += int(np.sum(prod > 0))
        disc += int(np.sum(prod < 0))
        ties_a += int(np.sum((da == 0) & (db != 0)))
        ties_b += int(np.sum((db == 0) & (da != 0)))
    denom = np.sqrt(float(conc + disc + ties_a) * float(conc + disc + ties_b))
    return (conc - disc) / denom if denom > 0 else float("nan")
