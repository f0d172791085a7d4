"""2^D spin patching of the autoregressive model (oracle, float64) -- TEST
INFRASTRUCTURE ONLY.

What the paper states (Methods, model configurations and training settings;
SI Sec. IV, table of parameter statistics): for the Edwards-Anderson lattices
the L^D spins are cut into non-overlapping 2 x ... x 2 blocks of 2^D spins, each
block becomes one token, so the sequence has (L/2)^D positions and the token
table and output head have 2^(2^D) rows (16 in 2D, 256 in 3D).  The model is
the unpatched one otherwise: q(sigma) = prod_t p_t(tok_t | tok_<t), the token
fed at position t is start (row 0) at t = 0, else tok_{t-1}.  The printed
parameter counts with and without patching differ exactly by the token table
and head rows this implies (pinned in the parameter-count fixture).

Readings (the paper fixes none of these):
  * patch order: raster order of the patch coordinates P = (P_0, ..., P_{D-1}),
    last coordinate fastest, the same convention as the site order;
  * bit order inside a token: the patch's site at offset o in {0,1}^D (site
    coordinates 2 P_k + o_k) gives bit m = sum_k o_k 2^(D-1-k) of the token,
    with bit value (sigma + 1) / 2;
  * categorical draw from one uniform u per (sample, position), the sampler's
    Philox stream: the token is found by walking the vocabulary from the top,
    tok = the largest k >= 1 with u < sum_{j >= k} p_j, else 0, i.e. u < p_{V-1}
    gives V-1, else u < p_{V-1} + p_{V-2} gives V-2, and so on.  With V = 2 this is the
    binary rule s = +1 iff u < p(+1), so unpatched sampling is the special case.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

from . import network as net
from .philox import uniforms


def patch_sites(L: int, D: int) -> np.ndarray:
    """Site index of bit m of patch t, int64 [(L/2)^D, 2^D]."""
    if L % 2:
        raise ValueError("patching needs an even lattice side")
    P = L // 2
    out = np.empty((P ** D, 2 ** D), dtype=np.int64)
    for t, pc in enumerate(itertools.product(range(P), repeat=D)):
        for m, oc in enumerate(itertools.product(range(2), repeat=D)):
            site = 0
            for k in range(D):
                site = site * L + 2 * pc[k] + oc[k]
            out[t, m] = site
    return out


def spins_to_tokens(spins, L: int, D: int) -> np.ndarray:
    """+-1 spins [B, L^D] -> tokens [B, (L/2)^D] in [0, 2^(2^D))."""
    s = (np.asarray(spins, dtype=np.int64) + 1) // 2
    sites = patch_sites(L, D)
    w = np.int64(1) << np.arange(sites.shape[1], dtype=np.int64)
    return (s[:, sites] * w).sum(axis=2)


def tokens_to_spins(tok, L: int, D: int) -> np.ndarray:
    """Inverse of spins_to_tokens: tokens [B, T] -> int8 +-1 spins [B, L^D]."""
    tok = np.asarray(tok, dtype=np.int64)
    sites = patch_sites(L, D)
    bits = (tok[:, :, None] >> np.arange(sites.shape[1], dtype=np.int64)) & 1
    out = np.zeros((tok.shape[0], L ** D), dtype=np.int8)
    out[:, sites.reshape(-1)] = (2 * bits - 1).reshape(tok.shape[0], -1)
    return out


def input_tokens(tok: torch.Tensor) -> torch.Tensor:
    """Token fed at each position: start (0) at t = 0, else tok_{t-1}."""
    start = torch.zeros_like(tok[:, :1])
    return torch.cat([start, tok[:, :-1]], dim=1)


def logits_tokens(theta: torch.Tensor, cfg, tok) -> torch.Tensor:
    """Teacher-forced logits z [B, T, vocab] of a token sequence (cfg.n_spins = T)."""
    p = net.unflatten(theta, cfg)
    tok = torch.as_tensor(np.asarray(tok, dtype=np.int64))
    B, T = tok.shape
    if T != cfg.n_spins:
        raise ValueError("sequence length does not match the model")
    x = net.embed(p, cfg, input_tokens(tok), torch.arange(T))
    vis = net.visibility(T, cfg.window, cfg.prefix)
    for l in range(cfg.n_layers):
        x = net.block(p, l, cfg, x, vis)
    return x @ p["head.w"].T + p["head.b"]


def log_q_tokens(theta, cfg, tok, chunk: int = 64) -> np.ndarray:
    """ln q(tok) = sum_t log p_t(tok_t | tok_<t), float64 [B]."""
    th = net.as_theta(theta)
    tok = torch.as_tensor(np.asarray(tok, dtype=np.int64))
    outs = []
    with torch.no_grad():
        for b0 in range(0, tok.shape[0], chunk):
            tk = tok[b0:b0 + chunk]
            lp = torch.log_softmax(logits_tokens(th, cfg, tk), dim=-1)
            outs.append(torch.gather(lp, -1, tk.unsqueeze(-1)).squeeze(-1).sum(dim=1))
    return torch.cat(outs).numpy()


def grad_surrogate_tokens(theta, cfg, tok, c, chunk: int = 32) -> np.ndarray:
    """grad_theta sum_b c_b ln q(tok_b), float64 [n_params]: reverse mode through
    the token logits above (the REINFORCE gradient of a patched model, Eq. 18,
    is this with c_b the weights of Eq. 19)."""
    tok = torch.as_tensor(np.asarray(tok, dtype=np.int64))
    c = torch.as_tensor(np.asarray(c, dtype=np.float64))
    th = net.as_theta(theta, requires_grad=True)
    g = torch.zeros_like(th)
    for b0 in range(0, tok.shape[0], chunk):
        th.grad = None
        tk = tok[b0:b0 + chunk]
        lp = torch.log_softmax(logits_tokens(th, cfg, tk), dim=-1)
        lq = torch.gather(lp, -1, tk.unsqueeze(-1)).squeeze(-1).sum(dim=1)
        (c[b0:b0 + chunk] * lq).sum().backward()
        g += th.grad
    return g.detach().numpy()


def log_q_spins(theta, cfg, spins, L: int, D: int, chunk: int = 64) -> np.ndarray:
    """ln q of spin configurations under the patched model."""
    return log_q_tokens(theta, cfg, spins_to_tokens(spins, L, D), chunk)


def categorical_draw(p, u) -> np.ndarray:
    """Token from probabilities p [B, V] and uniforms u [B], walking from the top."""
    p = np.asarray(p, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    B, V = p.shape
    tok = np.zeros(B, dtype=np.int64)
    for b in range(B):
        acc = 0.0
        for k in range(V - 1, 0, -1):
            acc += p[b, k]
            if u[b] < acc:
                tok[b] = k
                break
    return tok


def sample(theta, cfg, batch: int, seed: int, stream: int, b0: int = 0, u=None):
    """Ancestral sampling of token sequences, recomputing the prefix at each
    position.  Returns (tokens int64 [B, T], ln q float64 [B])."""
    th = net.as_theta(theta)
    T = cfg.n_spins
    if u is None:
        u = uniforms(seed, stream, batch, T, b0)
    tok = np.zeros((batch, T), dtype=np.int64)
    logq = np.zeros(batch)
    with torch.no_grad():
        for t in range(T):
            z = logits_tokens(th, cfg, tok)[:, t]          # position t sees tokens < t only
            lp = torch.log_softmax(z, dim=-1).numpy()
            tok[:, t] = categorical_draw(np.exp(lp), u[:, t])
            logq += lp[np.arange(batch), tok[:, t]]
    return tok, logq
