"""Variational free energy, its REINFORCE gradient and the parameter update (oracle, FP64).

F_q = (1/beta) sum_sigma q(sigma) [beta E(sigma) + ln q(sigma)]          (Eq. 5)
is estimated from B samples of q through the per-sample values
    f_b = (E_b + ln q_b / beta) / N,   F_q / N ~ mean_b f_b,
and its sample variance Var[f] = sum_b (f_b - mean)^2 / (B - 1) (the paper
reports "the variance of the estimated free energy" without a formula; this is
the reading used).

Gradient (Eqs. 16-19): with L_b = beta E_b + ln q_b and the baseline
Lbar = mean_b L_b, the estimator of grad F_q is
    g = 1/(beta B) sum_b (L_b - Lbar) grad ln q_b .
The paper writes the estimator "proportional to" this sum with 1/M; the factor
1/beta turns it into the gradient of F_q itself.  The surrogate whose gradient
is g is S(theta) = sum_b c_b ln q_b(theta) with c_b = (L_b - Lbar)/(beta B)
held fixed; its gradient is taken by reverse-mode differentiation of the FP64
network.
"""
from __future__ import annotations

import numpy as np
import torch

from . import network as net


def free_energy_stats(E, logq, beta: float, n: int):
    E = np.asarray(E, dtype=np.float64)
    logq = np.asarray(logq, dtype=np.float64)
    f = (E + logq / beta) / n
    mean = f.mean()
    var = ((f - mean) ** 2).sum() / (f.shape[0] - 1) if f.shape[0] > 1 else 0.0
    return float(mean), float(var)


def reinforce_weights(E, logq, beta: float):
    E = np.asarray(E, dtype=np.float64)
    logq = np.asarray(logq, dtype=np.float64)
    L = beta * E + logq
    return (L - L.mean()) / (beta * L.shape[0])


def surrogate(theta_t: torch.Tensor, cfg, spins, c) -> torch.Tensor:
    lq = net.log_q(theta_t, cfg, spins)
    return (torch.as_tensor(np.asarray(c, dtype=np.float64)) * lq).sum()


def grad_surrogate(theta, cfg, spins, c, chunk: int = 32) -> np.ndarray:
    """grad_theta sum_b c_b ln q_b(theta), float64 [n_params]."""
    spins = np.asarray(spins)
    c = np.asarray(c, dtype=np.float64)
    th = net.as_theta(theta, requires_grad=True)
    g = torch.zeros_like(th)
    for b0 in range(0, spins.shape[0], chunk):
        th.grad = None
        s = surrogate(th, cfg, spins[b0:b0 + chunk], c[b0:b0 + chunk])
        s.backward()
        g += th.grad
    return g.detach().numpy()


def reinforce_gradient(theta, cfg, spins, E, logq, beta: float) -> np.ndarray:
    return grad_surrogate(theta, cfg, spins, reinforce_weights(E, logq, beta))


def adam_update(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9,
                beta2: float = 0.999, eps: float = 1e-8, weight_decay: float = 0.0):
    """One Adam step (Kingma & Ba) with bias correction; step counts from 1.
    Returns (theta, m, v) as float64 arrays.  The paper's default optimiser is
    Muon (oracle.muon); Adam is the alternative it is compared with (Methods, optimiser comparison)."""
    g = np.asarray(grad, np.float64) + weight_decay * np.asarray(theta, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    theta = np.asarray(theta, np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
