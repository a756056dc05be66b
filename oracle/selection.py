"""Closed "interval" form of the quantile-Gaussian selection of Algorithm 1.

With full transmittance T_i before entry i and T_{i+1} = T_i (1 - alpha'_i),
Algorithm 1 keeps the count k equal to the number of thresholds
t_m = 1 - m/(K+1) lying strictly above the current T (the if/while pair
consumes every threshold a step crosses). Entry i is therefore selected
exactly when some threshold lies in the half-open interval
(T_{i+1}, T_i]:  T_{i+1} < t_m <= T_i, and the walk ends after the first
entry whose T_{i+1} falls below 1/(K+1).

This is a second, loop-free statement of the same selection; tests check it
against the step-by-step renderer on many random rays.
"""

from __future__ import annotations

import numpy as np


def interval_selection(alphas, K: int):
    """Indices (into ``alphas``) of the selected entries, in ray order."""
    a = np.asarray(alphas, dtype=np.float64)
    if a.size == 0:
        return []
    T_after = np.cumprod(1.0 - a)
    T_before = np.concatenate([[1.0], T_after[:-1]])
    below = np.nonzero(T_after < 1.0 / (K + 1.0))[0]
    last = int(below[0]) if below.size else a.size - 1
    t = np.array([1.0 - m / (K + 1.0) for m in range(1, K + 1)])
    sel = []
    for i in range(last + 1):
        if np.any((T_after[i] < t) & (t <= T_before[i])):
            sel.append(i)
    return sel
