"""The FlashVAN network q_theta in float64 (oracle).

What it computes, with the paper's notation:
  * tokens: s = (sigma + 1) / 2 in {0, 1}; the token table row s is the spin
    embedding (d_token = 2) and row 0 doubles as the start token (Alg. 2 feeds a
    start token 0 at the first step).
  * input of position t: x_t = [ T[tok_t] ; P[t] ]  (concatenated positional
    embedding, Eq. 15) with tok_0 = start and tok_t = s_{t-1}, so position t
    predicts site t from sites < t (Alg. 2: the token fed at step t is the one
    sampled at step t-1).
  * each decoder block (pre-LayerNorm wiring of Alg. 2):
        h <- h + concat_heads( softmax_j(q_t . k_j / sqrt(d_h)) v_j )   (Eqs. 2-3)
        h <- h + W2 GELU(W1 LN2(h) + b1) + b2
    with q, k, v = W_qkv LN1(h) + b_qkv, and no output projection W_O (the
    heads' concatenation is added to the residual directly, Eq. 3 and text).
  * attention mask: key j is visible from query t iff j <= t and
    (t - j <= W or j < P); W >= N-1, P = 0 is full causal attention, P = 0 is
    the plain sliding window of SI Eq. (S1).
  * head: z_t = W_h h_t + b_h, log p_t(s) = z_{t,s} - logsumexp(z_t) and
    ln q(sigma) = sum_t log p_t(s_t) (Alg. 1).
LayerNorm: affine, population variance, eps = 1e-5.  GELU: x Phi(x) with the
exact error function.  Neither is fixed by the paper (readings listed in the
design notes); the parameter counts the paper prints pin the affine LayerNorms,
the biased 4d-wide FFN, the biased QKV and the absence of W_O.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np
import torch

LN_EPS = 1e-5


def layout(cfg):
    """Ordered (name, shape) list of the flat parameter vector."""
    d = cfg.d_model
    out = [("tok_emb", (cfg.vocab, cfg.d_token)), ("pos_emb", (cfg.n_spins, d - cfg.d_token))]
    for l in range(cfg.n_layers):
        out += [(f"l{l}.ln1.g", (d,)), (f"l{l}.ln1.b", (d,)),
                (f"l{l}.qkv.w", (3 * d, d)), (f"l{l}.qkv.b", (3 * d,)),
                (f"l{l}.ln2.g", (d,)), (f"l{l}.ln2.b", (d,)),
                (f"l{l}.ffn1.w", (4 * d, d)), (f"l{l}.ffn1.b", (4 * d,)),
                (f"l{l}.ffn2.w", (d, 4 * d)), (f"l{l}.ffn2.b", (d,))]
    out += [("head.w", (cfg.vocab, d)), ("head.b", (cfg.vocab,))]
    return out


def count(cfg) -> int:
    return sum(int(np.prod(s)) for _, s in layout(cfg))


def unflatten(theta: torch.Tensor, cfg) -> Dict[str, torch.Tensor]:
    out, off = {}, 0
    for name, shape in layout(cfg):
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].view(*shape)
        off += n
    if off != theta.numel():
        raise ValueError(f"parameter vector has {theta.numel()} entries, layout needs {off}")
    return out


def as_theta(theta, requires_grad: bool = False) -> torch.Tensor:
    t = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone()
    return t.requires_grad_(requires_grad)


def visibility(n: int, window: int, prefix: int) -> torch.Tensor:
    t = torch.arange(n)[:, None]
    j = torch.arange(n)[None, :]
    return (j <= t) & ((t - j <= window) | (j < prefix))


def layer_norm(x, g, b):
    mu = x.mean(dim=-1, keepdim=True)
    var = ((x - mu) ** 2).mean(dim=-1, keepdim=True)
    return (x - mu) / torch.sqrt(var + LN_EPS) * g + b


def gelu(x):
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def tokens(spins: torch.Tensor) -> torch.Tensor:
    """Token fed at each position: start (0) at t = 0, else s_{t-1} = (sigma_{t-1}+1)/2."""
    s = (spins.long() + 1) // 2
    start = torch.zeros_like(s[:, :1])
    return torch.cat([start, s[:, :-1]], dim=1)


def embed(p, cfg, tok: torch.Tensor, positions: torch.Tensor) -> torch.Tensor:
    te = p["tok_emb"][tok]                       # [..., d_token]
    pe = p["pos_emb"][positions]                  # [..., d_pos]
    pe = pe.expand(*te.shape[:-1], pe.shape[-1])
    return torch.cat([te, pe], dim=-1)


def split_heads(x, n_heads):
    B, T, d = x.shape
    return x.view(B, T, n_heads, d // n_heads).transpose(1, 2)     # [B, H, T, dh]


def masked_attention(q, k, v, vis, n_heads):
    """q [B, T, d], k, v [B, J, d], vis [T, J] bool -> concat of head outputs [B, T, d]."""
    qh, kh, vh = split_heads(q, n_heads), split_heads(k, n_heads), split_heads(v, n_heads)
    dh = qh.shape[-1]
    s = torch.matmul(qh, kh.transpose(-1, -2)) / math.sqrt(dh)
    s = s.masked_fill(~vis, float("-inf"))
    w = torch.softmax(s, dim=-1)
    o = torch.matmul(w, vh)                                          # [B, H, T, dh]
    B, H, T, _ = o.shape
    return o.transpose(1, 2).reshape(B, T, H * dh)


def block(p, l, cfg, x, vis):
    d = cfg.d_model
    a = layer_norm(x, p[f"l{l}.ln1.g"], p[f"l{l}.ln1.b"])
    qkv = a @ p[f"l{l}.qkv.w"].T + p[f"l{l}.qkv.b"]
    q, k, v = qkv[..., :d], qkv[..., d:2 * d], qkv[..., 2 * d:]
    x = x + masked_attention(q, k, v, vis, cfg.n_heads)
    a2 = layer_norm(x, p[f"l{l}.ln2.g"], p[f"l{l}.ln2.b"])
    hdn = gelu(a2 @ p[f"l{l}.ffn1.w"].T + p[f"l{l}.ffn1.b"])
    return x + hdn @ p[f"l{l}.ffn2.w"].T + p[f"l{l}.ffn2.b"]


def logits(theta: torch.Tensor, cfg, spins) -> torch.Tensor:
    """Teacher-forced logits z [B, N, vocab] for the given spins (Alg. 1)."""
    p = unflatten(theta, cfg)
    spins = torch.as_tensor(np.asarray(spins))
    B, N = spins.shape
    if N != cfg.n_spins:
        raise ValueError("spin length does not match the model")
    x = embed(p, cfg, tokens(spins), torch.arange(N))
    vis = visibility(N, cfg.window, cfg.prefix)
    for l in range(cfg.n_layers):
        x = block(p, l, cfg, x, vis)
    return x @ p["head.w"].T + p["head.b"]


def log_p_sites(theta, cfg, spins, chunk: int = 64) -> torch.Tensor:
    """log p_t(s_t | s_<t) for every site, float64 [B, N]."""
    spins = torch.as_tensor(np.asarray(spins))
    outs = []
    for b0 in range(0, spins.shape[0], chunk):
        sp = spins[b0:b0 + chunk]
        z = logits(theta, cfg, sp)
        lp = torch.log_softmax(z, dim=-1)
        s = ((sp.long() + 1) // 2).unsqueeze(-1)
        outs.append(torch.gather(lp, -1, s).squeeze(-1))
    return torch.cat(outs, dim=0)


def log_q(theta, cfg, spins, chunk: int = 64) -> torch.Tensor:
    """ln q_theta(sigma) = sum_t log p_t(s_t), float64 [B]."""
    return log_p_sites(theta, cfg, spins, chunk).sum(dim=1)


def cond_plus(theta, cfg, spins, chunk: int = 64) -> torch.Tensor:
    """p_t(s_t = +1 | the given s_<t), teacher forced, float64 [B, N]."""
    spins = torch.as_tensor(np.asarray(spins))
    outs = []
    for b0 in range(0, spins.shape[0], chunk):
        z = logits(theta, cfg, spins[b0:b0 + chunk])
        outs.append(torch.softmax(z, dim=-1)[..., 1])
    return torch.cat(outs, dim=0)
