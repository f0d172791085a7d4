"""Flat FP32 parameter vector: its documented layout and seeded initial values.

Layout (row-major tensors, concatenated in this order):
  tok_emb [vocab, d_token]          token table; row 0 also serves as the start token
  pos_emb [n_spins, d_pos]          one row per sequence position
  per layer l = 0 .. n_layers-1:
    ln1.g [d], ln1.b [d]
    qkv.w [3d, d], qkv.b [3d]       rows 0..d-1 = Q, d..2d-1 = K, 2d..3d-1 = V;
                                    head h owns rows h*d_head .. (h+1)*d_head-1 of each
    ln2.g [d], ln2.b [d]
    ffn1.w [4d, d], ffn1.b [4d]
    ffn2.w [d, 4d], ffn2.b [d]
  head.w [vocab, d], head.b [vocab]
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .configs import ModelConfig


def param_layout(cfg: ModelConfig) -> List[Tuple[str, Tuple[int, ...], int]]:
    d = cfg.d_model
    out = []
    off = 0

    def add(name, shape):
        nonlocal off
        out.append((name, tuple(shape), off))
        off += int(np.prod(shape))

    add("tok_emb", (cfg.vocab, cfg.d_token))
    add("pos_emb", (cfg.n_spins, cfg.d_pos))
    for l in range(cfg.n_layers):
        add(f"l{l}.ln1.g", (d,))
        add(f"l{l}.ln1.b", (d,))
        add(f"l{l}.qkv.w", (3 * d, d))
        add(f"l{l}.qkv.b", (3 * d,))
        add(f"l{l}.ln2.g", (d,))
        add(f"l{l}.ln2.b", (d,))
        add(f"l{l}.ffn1.w", (4 * d, d))
        add(f"l{l}.ffn1.b", (4 * d,))
        add(f"l{l}.ffn2.w", (d, 4 * d))
        add(f"l{l}.ffn2.b", (d,))
    add("head.w", (cfg.vocab, d))
    add("head.b", (cfg.vocab,))
    return out


def num_params(cfg: ModelConfig) -> int:
    name, shape, off = param_layout(cfg)[-1]
    return off + int(np.prod(shape))


def init_params(cfg: ModelConfig, seed: int, style: str = "default") -> np.ndarray:
    """Seeded FP32 parameters.

    style "default": unit LayerNorm gains, zero biases, fan-in scaled weights.
    style "random":  every entry random (gains near 1, biases near 0) so that a
                     wrong gain, bias or index shows up in a comparison.
    style "sharp":   "random" with the output head scaled by 10, which pushes the
                     conditionals towards 0 and 1.
    """
    rng = np.random.default_rng(seed)
    d = cfg.d_model
    theta = np.zeros(num_params(cfg), dtype=np.float64)
    rnd = style in ("random", "sharp")
    for name, shape, off in param_layout(cfg):
        size = int(np.prod(shape))
        leaf = name.split(".", 1)[-1] if name.startswith("l") and name[1].isdigit() else name
        if leaf in ("ln1.g", "ln2.g"):
            v = 1.0 + (0.1 * rng.standard_normal(size) if rnd else 0.0)
        elif leaf in ("ln1.b", "ln2.b", "qkv.b", "ffn1.b", "ffn2.b", "head.b"):
            v = 0.1 * rng.standard_normal(size) if rnd else np.zeros(size)
        elif leaf in ("tok_emb", "pos_emb"):
            v = rng.standard_normal(size)
        elif leaf == "qkv.w":
            v = rng.standard_normal(size) / np.sqrt(d)
        elif leaf == "ffn1.w":
            v = rng.standard_normal(size) / np.sqrt(d)
        elif leaf == "ffn2.w":
            v = rng.standard_normal(size) / np.sqrt(4 * d)
        elif leaf == "head.w":
            v = rng.standard_normal(size) / np.sqrt(d) * (10.0 if style == "sharp" else 1.0)
        else:
            raise KeyError(name)
        theta[off:off + size] = v
    return theta.astype(np.float32)
