"""Seeded disorder instances.

SK: couplings J_ij = J_ji with i < j drawn i.i.d. Gaussian of variance 1/N
(unit-variance draws pre-scaled by 1/sqrt(N)), zero diagonal.
EA: a D-dimensional hypercubic lattice of side L, sites in raster order (last
coordinate fastest), one bond per nearest-neighbour pair, bonds +/-1 with equal
probability or unit Gaussian.  Each unordered pair is listed exactly once.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class Instance:
    n: int
    edges_i: np.ndarray           # int32 [E]
    edges_j: np.ndarray           # int32 [E]
    J: np.ndarray                 # float64 [E]  (integer valued for +/-J)
    bonds: str                    # "pm1" | "gauss"
    dense: Optional[np.ndarray] = None   # float64 [N, N] for SK (symmetric, zero diagonal)
    L: int = 0
    dim: int = 0
    pbc: bool = True

    @property
    def n_edges(self) -> int:
        return int(self.edges_i.shape[0])


def sk_instance(n: int, seed: int) -> Instance:
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    upper = np.triu(g, 1) / np.sqrt(n)
    dense = upper + upper.T
    ii, jj = np.triu_indices(n, 1)
    return Instance(n=n, edges_i=ii.astype(np.int32), edges_j=jj.astype(np.int32),
                    J=dense[ii, jj].copy(), bonds="gauss", dense=dense)


def lattice_edges(L: int, dim: int, pbc: bool = True):
    """Nearest-neighbour pairs (i, i + e_k) of an L^dim lattice in raster order."""
    n = L ** dim
    coords = np.stack(np.unravel_index(np.arange(n), (L,) * dim), axis=1)
    ei, ej = [], []
    for site in range(n):
        c = coords[site]
        for k in range(dim):
            nc = c.copy()
            nc[k] += 1
            if nc[k] == L:
                if not pbc:
                    continue
                nc[k] = 0
            ei.append(site)
            ej.append(int(np.ravel_multi_index(tuple(nc), (L,) * dim)))
    return np.asarray(ei, np.int32), np.asarray(ej, np.int32)


def patch_edges(L: int, dim: int, pbc: bool = True):
    """Interaction graph of the (L/2)^dim patches of 2^dim sites (patches in raster
    order of their coordinates): two patches are joined if any of their sites are
    lattice neighbours.  Returns (n_patches, pi, pj), each pair once, pi < pj."""
    if L % 2:
        raise ValueError("patches need an even lattice side")
    n = L ** dim
    coords = np.stack(np.unravel_index(np.arange(n), (L,) * dim), axis=1)
    owner = np.ravel_multi_index(tuple((coords // 2).T), (L // 2,) * dim)
    ei, ej = lattice_edges(L, dim, pbc)
    a, b = owner[ei], owner[ej]
    keep = a != b
    pairs = np.unique(np.sort(np.stack([a[keep], b[keep]], 1), axis=1), axis=0)
    return (L // 2) ** dim, pairs[:, 0].astype(np.int32), pairs[:, 1].astype(np.int32)


def ea_instance(L: int, dim: int, seed: int, bonds: str = "pm1", pbc: bool = True) -> Instance:
    if pbc and L < 3:
        raise ValueError("periodic lattices need L >= 3 (L = 2 would list a pair twice)")
    ei, ej = lattice_edges(L, dim, pbc)
    rng = np.random.default_rng(seed)
    if bonds == "pm1":
        J = rng.integers(0, 2, size=ei.shape[0]).astype(np.float64) * 2.0 - 1.0
    elif bonds == "gauss":
        J = rng.standard_normal(ei.shape[0])
    else:
        raise ValueError(bonds)
    return Instance(n=L ** dim, edges_i=ei, edges_j=ej, J=J, bonds=bonds, L=L, dim=dim, pbc=pbc)


def chain_instance(n: int, J: float = 1.0) -> Instance:
    """Open 1D chain with uniform bond J between consecutive sites."""
    ei = np.arange(n - 1, dtype=np.int32)
    return Instance(n=n, edges_i=ei, edges_j=ei + 1, J=np.full(n - 1, float(J)),
                    bonds="gauss", L=n, dim=1, pbc=False)


def random_spins(batch: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 2, size=(batch, n)) * 2 - 1).astype(np.int8)
