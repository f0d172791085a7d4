"""Overlap distribution and the annealing schedule (oracle) -- TEST
INFRASTRUCTURE ONLY.

Overlap (Eq. overlap_distribution): two independent replicas s^1, s^2 at the
same temperature have q = (1/N) sum_i s^1_i s^2_i.  The paper draws its p(q)
from pairs of independent samples; reading: every unordered pair {a, b}, a != b,
of a batch of independent samples is one pair of replicas, and the histogram
counts pairs by their number of agreeing sites k = (N + N q) / 2, k = 0..N
(q = 2k/N - 1).  Integer arithmetic: exact.

Annealing (Methods, variational annealing): with T_0, n_warmup, n_eq and
n_anneal,
    T_i = T_0                                                  i <= n_warmup
    T_i = T_0 - (T_0 / n_anneal) floor((i - n_warmup) / n_eq)  i >  n_warmup,
reaching T = 0 at i = n_warmup + n_eq n_anneal, the paper's total step count.
Reading: the floor is capped at n_anneal, so T stays at 0 afterwards (a step
at T = 0 has no finite beta; callers stop before it).
"""
from __future__ import annotations

import math

import numpy as np


def overlap_counts(spins) -> np.ndarray:
    """counts[k] = number of pairs a < b with k agreeing sites, int64 [N + 1]."""
    s = np.asarray(spins, dtype=np.int64)
    B, N = s.shape
    Q = s @ s.T
    a, b = np.triu_indices(B, k=1)
    k = (Q[a, b] + N) // 2
    return np.bincount(k, minlength=N + 1).astype(np.int64)


def anneal_temperature(i: int, T0: float, n_warmup: int, n_eq: int, n_anneal: int) -> float:
    if i <= n_warmup:
        return float(T0)
    k = min((i - n_warmup) // n_eq, n_anneal)
    return float(T0 - (T0 / n_anneal) * k)
