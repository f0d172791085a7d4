"""Local Monte Carlo refinement and the self-distillation gradient weights
(oracle, float64) -- TEST INFRASTRUCTURE ONLY.

What the paper states (Results, 3D EA; Methods, training strategy; SI Sec.
I C): samples drawn from q_theta are refined by a short local Monte Carlo
trajectory before the loss is evaluated, and the gradient of Eq. (loss2) adds
a likelihood term,
    grad ~ (1/M) sum_m (L(s_m) - Lbar) grad ln q(s_m)  -  w grad ln q(s_m),
evaluated on the refined samples s_m, with L = beta E + ln q.  The paper names
neither the Monte Carlo move, the number of sweeps nor w; the readings here:

  * Metropolis single-spin flips at inverse temperature beta, in checkerboard
    order: every sweep updates the sites of colour 0, then those of colour 1.
    Within a half-sweep every site's local field h_i = sum_j J_ij s_j is taken
    from the configuration at the start of the half-sweep; with a proper
    2-colouring (a bipartite lattice: periodic boundaries need even L) no two
    sites of one colour interact, so each half-sweep is exact sequential
    single-site Metropolis.  Flipping s_i changes E = -sum_(ij) J_ij s_i s_j
    by dE = 2 s_i h_i; the flip is accepted iff u < exp(-beta dE).
  * The uniform u of (sample b, sweep k, site i) is Philox4x32-10 with key
    (seed mod 2^32, seed >> 32), counter (i >> 2, b, k, stream), word i & 3,
    u = (word >> 8) 2^-24 -- the sampler's generator with the sweep index and a
    32-bit stream tag in the last two counter words.
  * Weights: c_m = ((L_m - Lbar) - w) / (beta M): Eq. (loss2) is
    (1/M) sum_m ((L - Lbar) - w) grad ln q_m up to a constant factor, and the
    factor is taken to be the 1/beta of the exact grad F_q estimator
    (estimator.py, Eq. 18), applied to both terms, so that with w = 0 these are
    its REINFORCE weights.  Lbar is the batch mean of L over the refined samples; ln q of a
    refined sample is its teacher-forced log-likelihood.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32_10


def checkerboard_colour(L: int, dim: int) -> np.ndarray:
    """Colour (sum of raster coordinates mod 2) of each site, last coordinate fastest."""
    idx = np.arange(L ** dim)
    c = np.zeros(L ** dim, dtype=np.int64)
    for _ in range(dim):
        c += idx % L
        idx //= L
    return (c % 2).astype(np.int8)


def neighbours(n: int, edges_i, edges_j, J):
    """Full adjacency (both directions) of the pair list: lists of (j, J_ij) per site."""
    adj = [[] for _ in range(n)]
    for a, b, v in zip(np.asarray(edges_i), np.asarray(edges_j), np.asarray(J, dtype=np.float64)):
        adj[int(a)].append((int(b), float(v)))
        adj[int(b)].append((int(a), float(v)))
    return adj


def lmc_uniforms(seed: int, stream: int, batch: int, n: int, sweep: int, b0: int = 0) -> np.ndarray:
    """u[b, i] of one sweep, float64 [batch, n]."""
    nb = (n + 3) // 4
    b = np.arange(b0, b0 + batch, dtype=np.uint64)[:, None]
    g = np.arange(nb, dtype=np.uint64)[None, :]
    ctr = np.empty((batch, nb, 4), dtype=np.uint64)
    ctr[..., 0] = g
    ctr[..., 1] = b
    ctr[..., 2] = np.uint64(sweep & 0xFFFFFFFF)
    ctr[..., 3] = np.uint64(stream & 0xFFFFFFFF)
    key = np.empty((batch, nb, 2), dtype=np.uint64)
    key[..., 0] = np.uint64(seed & 0xFFFFFFFF)
    key[..., 1] = np.uint64((seed >> 32) & 0xFFFFFFFF)
    words = philox4x32_10(ctr, key).reshape(batch, nb * 4)[:, :n]
    return (words >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def local_fields(spins, adj) -> np.ndarray:
    s = np.asarray(spins, dtype=np.float64)
    h = np.zeros_like(s)
    for i, nb in enumerate(adj):
        for j, v in nb:
            h[:, i] += v * s[:, j]
    return h


def metropolis_checkerboard(spins, adj, colour, beta: float, sweeps: int, seed: int, stream: int, b0: int = 0,
                            uniforms=None, margins: bool = False):
    """Refined copy of spins (int8 +-1 [batch, n]) after `sweeps` checkerboard sweeps.
    Returns (spins, accepted flips per sample), plus with margins=True the
    smallest |u - exp(-beta dE)| per sample over its decisions with
    exp(-beta dE) < 1 (how close a decision came to the other outcome).
    uniforms(sweep) -> [batch, n] may replace the Philox draw (tests)."""
    s = np.array(spins, dtype=np.int64)
    batch, n = s.shape
    colour = np.asarray(colour)
    acc = np.zeros(batch, dtype=np.int64)
    marg = np.full(batch, np.inf)
    for k in range(sweeps):
        u = uniforms(k) if uniforms is not None else lmc_uniforms(seed, stream, batch, n, k, b0)
        for c in (0, 1):
            h = local_fields(s, adj)
            dE = 2.0 * s * h
            mine = colour[None, :] == c
            with np.errstate(over="ignore"):
                p = np.exp(-beta * dE)
            flip = (u < p) & mine
            if margins:
                d = np.where(mine & (p < 1.0), np.abs(u - p), np.inf)
                marg = np.minimum(marg, d.min(axis=1))
            s = np.where(flip, -s, s)
            acc += flip.sum(axis=1)
    if margins:
        return s.astype(np.int8), acc, marg
    return s.astype(np.int8), acc


def distill_weights(E, logq, beta: float, w: float) -> np.ndarray:
    """c_m = ((L_m - Lbar) - w) / (beta M), L = beta E + ln q (float64)."""
    L = beta * np.asarray(E, dtype=np.float64) + np.asarray(logq, dtype=np.float64)
    M = L.shape[0]
    return ((L - L.mean()) - w) / (beta * M)
