"""Ordered Markov boundary and the attention mask it implies (oracle).

Methods, "Autoregressive factorization and the ordered Markov boundary": with
sites ordered by index, P_i = {j < i} (past) and F_i = {j > i} (future), the
ordered Markov boundary of i is the set of past sites that are adjacent to i
or joined to i by a path whose inner nodes all lie in F_i (Eqs. 11-13).  The
autoregressive conditional of sigma_i depends on the past only through it.

Mask rule (SI Sec. I A, with the boundary-condition reading used here):
position p carries the token of site p-1 and predicts site p, so site j < i is
available to the query that predicts i iff position j+1 is visible from
position i.  The paper's window is A_ij = 0 for i - j > W with W >= d_max
(SI Eq. S1), W measured in sites.  Under periodic boundaries the first row
(plane) stays in the boundary of the last one, so the band alone is not exact;
the rule adds a prefix of always-visible positions:
  for each candidate prefix P = 0..N, W(P) is the largest site distance i - j
  over boundary pairs (i, j) not covered by the prefix (j + 1 >= P), and the
  chosen (P, W) minimises P + W, the smallest P winning ties.
Open lattices give P = 0, W = L^(D-1); periodic ones P = L^(D-1) + 1,
W = L^(D-1); the complete SK graph gives full causal attention, W = N - 1.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from .physics import all_configs


def adjacency(n, ei, ej):
    adj = [set() for _ in range(n)]
    for a, b in zip(np.asarray(ei).tolist(), np.asarray(ej).tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def ordered_boundary(n, ei, ej):
    """List of sorted boundary sets, one per site, by search through future sites."""
    adj = adjacency(n, ei, ej)
    out = []
    for i in range(n):
        seen = {i}
        dq = deque([i])
        past = set()
        while dq:
            v = dq.popleft()
            for w in adj[v]:
                if w < i:
                    past.add(w)
                elif w > i and w not in seen:
                    seen.add(w)
                    dq.append(w)
        out.append(sorted(past))
    return out


def derive_mask(n, ei, ej):
    """(window W, prefix P) by the rule in the module docstring."""
    bnd = ordered_boundary(n, ei, ej)
    # far[j] = largest distance i - j over boundary pairs whose past site is j
    far = np.zeros(n + 1, dtype=np.int64)
    for i in range(n):
        for j in bnd[i]:
            far[j] = max(far[j], i - j)
    best = None
    for P in range(n + 1):
        # pairs not covered by a prefix P are those with j >= P - 1
        W = int(far[max(P - 1, 0):].max()) if P - 1 < n else 0
        cost = P + W
        if best is None or cost < best[0]:
            best = (cost, W, P)
    return best[1], best[2]


def mask_covers(n, bnd, window, prefix) -> bool:
    for i in range(n):
        for j in bnd[i]:
            pos = j + 1
            if not (pos <= i and (i - pos <= window or pos < prefix)):
                return False
    return True


def brute_force_dependence(n, ei, ej, J, beta):
    """For every site i, the set of past sites the exact Boltzmann conditional
    P(sigma_i = +1 | sigma_<i) actually depends on, found by enumeration
    (Eq. 13: marginalise the future, then compare prefixes that differ at one site)."""
    sig = all_configs(n).astype(np.float64)
    E = -(sig[:, ei] * sig[:, ej] * np.asarray(J)[None, :]).sum(axis=1)
    w = np.exp(-beta * (E - E.min()))
    deps = []
    for i in range(n):
        m = w.reshape(2 ** i, 2, 2 ** (n - i - 1)).sum(axis=2)      # [prefix, sigma_i]
        cond = m[:, 1] / m.sum(axis=1)                              # P(+1 | prefix)
        dep = []
        for j in range(i):
            bit = 1 << (i - 1 - j)                                   # site j's bit in the prefix index
            idx = np.arange(2 ** i)
            lo = idx[(idx & bit) == 0]
            if np.max(np.abs(cond[lo] - cond[lo | bit])) > 1e-10:
                dep.append(j)
        deps.append(dep)
    return deps
