"""Spin energies and exact thermodynamics by enumeration (oracle, FP64).

Energy: E(sigma) = - sum over interacting pairs {i, j}, each unordered pair
counted once, of J_ij sigma_i sigma_j.  For SK the pair sum runs over i < j
with J_ij of variance 1/N (Eq. 6: unit-variance bonds with the 1/sqrt(N)
prefactor folded into J); for EA it runs over nearest-neighbour pairs (Eq. 8).
"""
from __future__ import annotations

import numpy as np


def energy_edges(spins: np.ndarray, ei: np.ndarray, ej: np.ndarray, J: np.ndarray) -> np.ndarray:
    """E_b = -sum_e J_e s_{b, i_e} s_{b, j_e}, float64 [B]."""
    s = spins.astype(np.float64)
    return -(s[:, ei] * s[:, ej] * J[None, :]).sum(axis=1)


def energy_edges_int(spins: np.ndarray, ei: np.ndarray, ej: np.ndarray, J: np.ndarray) -> np.ndarray:
    """Exact integer energy for integer bonds (+/-J), int64 [B]."""
    Ji = np.rint(J).astype(np.int64)
    if not np.array_equal(Ji.astype(np.float64), J):
        raise ValueError("bonds are not integers")
    s = spins.astype(np.int64)
    return -(s[:, ei] * s[:, ej] * Ji[None, :]).sum(axis=1)


def energy_dense(spins: np.ndarray, Jd: np.ndarray) -> np.ndarray:
    """SK form: -sum_{i<j} J_ij s_i s_j = -1/2 s^T J s for symmetric J, zero diagonal."""
    s = spins.astype(np.float64)
    return -0.5 * np.einsum("bi,ij,bj->b", s, Jd, s)


def all_configs(n: int) -> np.ndarray:
    """Every sigma in {-1, +1}^n, int8 [2^n, n]; site 0 is the most significant bit."""
    idx = np.arange(2 ** n, dtype=np.int64)[:, None]
    bits = (idx >> np.arange(n - 1, -1, -1, dtype=np.int64)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)


def log_partition(energies: np.ndarray, beta: float) -> float:
    """ln Z = ln sum exp(-beta E) by log-sum-exp over an enumerated energy list."""
    a = -beta * energies
    m = a.max()
    return float(m + np.log(np.exp(a - m).sum()))


def free_energy_exact(energies: np.ndarray, beta: float) -> float:
    """F = -(1/beta) ln Z (Results, Framework)."""
    return -log_partition(energies, beta) / beta
