"""Ancestral sampling through q_theta (oracle, FP64).

kv_sample follows the KV-cache procedure of Alg. 2 (Methods, sampling
strategy): at step t only the new q_t, k_t, v_t are computed per layer, k_t and
v_t are appended to the layer's cache, and the query attends to the visible
cached keys including its own (append-then-attend: the attention sum of Eq. 3
runs up to j = t).  The head gives p_t, a uniform u(b, t) from the Philox
stream decides s_t = +1 iff u < p_t(+1) (strict), and ln q accumulates
log p_t(s_t).  The cache here keeps every position (no ring buffer): it is the
plain definition, the GPU's band ring is a storage detail.

naive_sample recomputes the whole teacher-forced network on the prefix at each
step (the O(N^3 d) procedure the KV cache replaces); both must give the same
spins.
"""
from __future__ import annotations

import numpy as np
import torch

from . import network as net
from .philox import uniforms


def kv_sample(theta, cfg, batch: int, seed: int, stream: int, b0: int = 0,
              u: np.ndarray | None = None):
    """Returns (spins int8 [B, N], log_q float64 [B], p_plus float64 [B, N])."""
    th = net.as_theta(theta)
    p = net.unflatten(th, cfg)
    N, d, H = cfg.n_spins, cfg.d_model, cfg.n_heads
    if u is None:
        u = uniforms(seed, stream, batch, N, b0)
    u = torch.as_tensor(u, dtype=torch.float64)
    vis = net.visibility(N, cfg.window, cfg.prefix)
    K = [torch.zeros(batch, N, d, dtype=torch.float64) for _ in range(cfg.n_layers)]
    V = [torch.zeros(batch, N, d, dtype=torch.float64) for _ in range(cfg.n_layers)]
    s = torch.zeros(batch, N, dtype=torch.long)
    logq = torch.zeros(batch, dtype=torch.float64)
    pplus = torch.zeros(batch, N, dtype=torch.float64)
    with torch.no_grad():
        for t in range(N):
            tok = torch.zeros(batch, dtype=torch.long) if t == 0 else s[:, t - 1]
            h = net.embed(p, cfg, tok, torch.tensor(t))              # [B, d]
            keys = torch.nonzero(vis[t]).flatten()                     # visible key positions
            for l in range(cfg.n_layers):
                a = net.layer_norm(h, p[f"l{l}.ln1.g"], p[f"l{l}.ln1.b"])
                qkv = a @ p[f"l{l}.qkv.w"].T + p[f"l{l}.qkv.b"]
                q, k, v = qkv[:, :d], qkv[:, d:2 * d], qkv[:, 2 * d:]
                K[l][:, t] = k
                V[l][:, t] = v
                o = net.masked_attention(q[:, None, :], K[l][:, keys], V[l][:, keys],
                                         torch.ones(1, keys.numel(), dtype=torch.bool), H)
                h = h + o[:, 0]
                a2 = net.layer_norm(h, p[f"l{l}.ln2.g"], p[f"l{l}.ln2.b"])
                hdn = net.gelu(a2 @ p[f"l{l}.ffn1.w"].T + p[f"l{l}.ffn1.b"])
                h = h + hdn @ p[f"l{l}.ffn2.w"].T + p[f"l{l}.ffn2.b"]
            z = h @ p["head.w"].T + p["head.b"]
            lp = torch.log_softmax(z, dim=-1)
            pp = torch.softmax(z, dim=-1)[:, 1]
            st = (u[:, t] < pp).long()
            s[:, t] = st
            logq += torch.gather(lp, 1, st[:, None])[:, 0]
            pplus[:, t] = pp
    spins = (2 * s - 1).to(torch.int8).numpy()
    return spins, logq.numpy(), pplus.numpy()


def naive_sample(theta, cfg, batch: int, seed: int, stream: int, b0: int = 0):
    """Same draw as kv_sample, recomputing the full prefix at every step."""
    th = net.as_theta(theta)
    N = cfg.n_spins
    u = uniforms(seed, stream, batch, N, b0)
    spins = np.ones((batch, N), dtype=np.int8)
    logq = np.zeros(batch)
    with torch.no_grad():
        for t in range(N):
            z = net.logits(th, cfg, spins)[:, t]       # position t sees only tokens < t
            lp = torch.log_softmax(z, dim=-1).numpy()
            pp = torch.softmax(z, dim=-1)[:, 1].numpy()
            st = (u[:, t] < pp).astype(np.int64)
            spins[:, t] = (2 * st - 1).astype(np.int8)
            logq += lp[np.arange(batch), st]
    return spins, logq


def decision_check(theta, cfg, spins, seed: int, stream: int, tol: float, b0: int = 0):
    """Teacher-forced decision check of GPU samples.

    For each sample and site, p_t(+1) is evaluated in float64 on the sample's own
    prefix; the site must satisfy s_t = [u < p] wherever |u - p| >= tol.
    Returns (n_mismatch outside tol, n_exempt within tol, max |u - p| among mismatches).
    """
    spins = np.asarray(spins)
    B, N = spins.shape
    u = uniforms(seed, stream, B, N, b0)
    pp = net.cond_plus(net.as_theta(theta), cfg, spins).numpy()
    want = u < pp
    got = spins > 0
    close = np.abs(u - pp) < tol
    bad = (want != got) & ~close
    return int(bad.sum()), int(close.sum()), pp
