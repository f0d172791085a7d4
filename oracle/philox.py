"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), written from its published
definition, and the uniform draw the sampler uses.

One round maps counter (c0, c1, c2, c3) and key (k0, k1) to
  (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57; between rounds the key is bumped by the
Weyl constants (0x9E3779B9, 0xBB67AE85).  Ten rounds.

Draw used by ancestral sampling (the method only says "Categorical(p_t)",
Alg. 2; the generator is fixed here):
  key     = (seed mod 2^32, seed >> 32)
  counter = (t >> 2, b, stream mod 2^32, stream >> 32)
  u(b, t) = (word[t & 3] >> 8) * 2^-24        (exact in float32 and float64)
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: uint64 array [..., 4] of 32-bit words; key: uint64 array [..., 2]."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & MASK32 for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK32
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def uniforms(seed: int, stream: int, batch: int, n: int, b0: int = 0) -> np.ndarray:
    """u[b, t] for samples b0 .. b0+batch-1 and sites 0 .. n-1, float64 [batch, n]."""
    nb = (n + 3) // 4
    b = np.arange(b0, b0 + batch, dtype=np.uint64)[:, None]
    g = np.arange(nb, dtype=np.uint64)[None, :]
    ctr = np.empty((batch, nb, 4), dtype=np.uint64)
    ctr[..., 0] = g
    ctr[..., 1] = b
    ctr[..., 2] = np.uint64(stream & 0xFFFFFFFF)
    ctr[..., 3] = np.uint64((stream >> 32) & 0xFFFFFFFF)
    key = np.empty((batch, nb, 2), dtype=np.uint64)
    key[..., 0] = np.uint64(seed & 0xFFFFFFFF)
    key[..., 1] = np.uint64((seed >> 32) & 0xFFFFFFFF)
    words = philox4x32_10(ctr, key).reshape(batch, nb * 4)[:, :n]
    return (words >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
