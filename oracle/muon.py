"""Muon parameter update in float64 (oracle) -- TEST INFRASTRUCTURE ONLY.

What it computes (Methods, comparison of optimisers: the momentum /
orthogonalisation / step equations there):
    M_t = mu M_{t-1} + G_t                          momentum, M_0 = 0
    O_t = NewtonSchulz(M_t)                         approximate orthogonalisation
    W_t = W_{t-1} - eta ( s(W) O_t + lambda W_{t-1} )
The paper adds weight decay and RMS scale alignment from the Muon-at-scale work
it cites; there the update of an A x B matrix is scaled by 0.2 sqrt(max(A, B))
so that its RMS matches a typical Adam update.  Here s(W) = rms_scale *
sqrt(max(rows, cols)), rms_scale = 0.2 by default.

Newton-Schulz, as published with the Muon optimiser the paper cites (the
paper prints no coefficients): X_0 = M / (||M||_F + eps); a wide X (rows <=
cols) is iterated as
    A = X X^T,   X <- a X + (b A + c A^2) X,   (a, b, c) = (3.4445, -4.7750, 2.0315),
and a tall matrix as its transpose.  Each iteration maps every singular value
x of X to p(x) = a x + b x^3 + c x^5 and keeps the singular vectors; that is
what the pins check.

Which parameters take Muon: the per-layer weight matrices W_qkv, W1 and W2.
Every other parameter (token and position tables, head, biases, LayerNorm
gains and shifts) takes the Adam step of estimator.adam_update, as in the
cited Muon references, which leave embeddings, output head and vectors to
Adam.  The paper does not say which parameters it orthogonalises.

State: one first-moment array m and one second-moment array v over the flat
parameter vector; on Muon entries m is the momentum M and v is unused.
"""
from __future__ import annotations

import math

import numpy as np

from . import network
from .estimator import adam_update

NS_COEFFS = (3.4445, -4.7750, 2.0315)
MATRIX_KINDS = ("qkv.w", "ffn1.w", "ffn2.w")


def newton_schulz(M, steps: int = 5, eps: float = 1e-7, coeffs=NS_COEFFS) -> np.ndarray:
    """NewtonSchulz(M) in float64, same shape as M."""
    X = np.array(M, dtype=np.float64)
    if X.ndim != 2:
        raise ValueError("Newton-Schulz takes a matrix")
    X = X / (np.linalg.norm(X) + eps)
    tall = X.shape[0] > X.shape[1]
    if tall:
        X = X.T
    a, b, c = coeffs
    for _ in range(steps):
        A = X @ X.T
        B = b * A + c * (A @ A)
        X = a * X + B @ X
    return X.T if tall else X


def is_muon_param(name: str) -> bool:
    return name.split(".", 1)[-1] in MATRIX_KINDS


def muon_entries(cfg) -> np.ndarray:
    """Boolean mask over the flat parameter vector: True where Muon applies."""
    mask, off = np.zeros(network.count(cfg), dtype=bool), 0
    for name, shape in network.layout(cfg):
        n = int(np.prod(shape))
        if is_muon_param(name):
            mask[off:off + n] = True
        off += n
    return mask


def muon_update(theta, grad, m, v, step: int, cfg, lr: float, momentum: float = 0.95,
                weight_decay: float = 0.0, rms_scale: float = 0.2, ns_steps: int = 5, ns_eps: float = 1e-7,
                adam_lr: float = 1e-3, adam_beta1: float = 0.9, adam_beta2: float = 0.999, adam_eps: float = 1e-8,
                adam_weight_decay: float = 0.0):
    """One Muon step over the flat parameter vector; returns (theta, m, v) in float64."""
    theta = np.array(theta, dtype=np.float64)
    grad = np.asarray(grad, dtype=np.float64)
    m = np.array(m, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    off = 0
    for name, shape in network.layout(cfg):
        n = int(np.prod(shape))
        sl = slice(off, off + n)
        if is_muon_param(name):
            M = momentum * m[sl] + grad[sl]
            m[sl] = M
            O = newton_schulz(M.reshape(shape), ns_steps, ns_eps)
            scale = rms_scale * math.sqrt(max(shape))
            theta[sl] = theta[sl] - lr * (scale * O.ravel() + weight_decay * theta[sl])
        else:
            theta[sl], m[sl], v[sl] = adam_update(theta[sl], grad[sl], m[sl], v[sl], step, adam_lr, adam_beta1,
                                                  adam_beta2, adam_eps, adam_weight_decay)
        off += n
    return theta, m, v
