"""The paper's parallel processing scheme, FP64.  Test infrastructure only.

Section "Simulating live and parallel processing": the data are split into
disjoint subsets; every subset is iterated independently for a few
iterations, starting from the shared object and illumination, and then the
object and the illumination are averaged over the subsets (a hybrid between
sequential ePIE and batch methods).  The paper notes that the result depends
on the number of subsets and does not reproduce sequential ePIE.
"""
from __future__ import annotations

import numpy as np

from .epie import reconstruct


def subset_round(obj, probe, positions, intensities, subsets, schedules, alpha=1.0, beta=1.0,
                 dtype=np.complex128):
    """One round: subset k (an index array into the full position list) runs
    the sweeps schedules[k] = [(order, offsets or None), ...] (orders index
    the subset's own positions) from (obj, probe); returns the means of the
    subsets' objects and probes, and each subset's running errors."""
    objs, probes, errs = [], [], []
    for sub, sched in zip(subsets, schedules):
        sub = np.asarray(sub, dtype=np.int64)
        O, P, e = reconstruct(obj, probe, np.asarray(positions)[sub], np.asarray(intensities)[sub], sched,
                              alpha, beta, dtype)
        objs.append(O)
        probes.append(P)
        errs.append(e)
    K = len(objs)
    O = objs[0].copy()
    P = probes[0].copy()
    for k in range(1, K):
        O = O + objs[k]
        P = P + probes[k]
    return O / K, P / K, errs


def round_robin(count, k):
    """Assign positions 0..count-1 (in acquisition order) to k subsets in
    turn, as the paper's live parallel experiment does."""
    return [np.arange(i, count, k, dtype=np.int64) for i in range(k)]
