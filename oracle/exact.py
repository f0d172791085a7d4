"""Exact quantities by enumerating all 2^N configurations (oracle, N <= 16).

sum_sigma q(sigma)                      must equal 1 for any theta (normalised
                                        autoregressive product, Eq. 1 / Eq. 11)
F   = -(1/beta) ln Z                    (Results, Framework)
F_q = (1/beta) sum q [beta E + ln q]    (Eq. 5), with F_q >= F  (Eq. 4)
grad F_q = (1/beta) E_q[(beta E + ln q) grad ln q]   (Eq. 18)
"""
from __future__ import annotations

import numpy as np
import torch

from . import network as net
from .physics import all_configs, free_energy_exact


def enumerate_logq(theta, cfg, chunk: int = 4096):
    sig = all_configs(cfg.n_spins)
    lq = net.log_q(net.as_theta(theta), cfg, sig, chunk=chunk).detach().numpy()
    return sig, lq


def exact_free_energies(theta, cfg, energies: np.ndarray, beta: float):
    """(F_q, F, sum q) with energies over all_configs order."""
    _, lq = enumerate_logq(theta, cfg)
    q = np.exp(lq)
    Fq = float((q * (beta * energies + lq)).sum() / beta)
    return Fq, free_energy_exact(energies, beta), float(q.sum())


def exact_grad_Fq(theta, cfg, energies: np.ndarray, beta: float, chunk: int = 4096) -> np.ndarray:
    """(1/beta) sum_sigma q (beta E + ln q) grad ln q, by reverse mode over the
    exact weighted sum with the weights q (beta E + ln q) held fixed."""
    sig = all_configs(cfg.n_spins)
    th = net.as_theta(theta, requires_grad=True)
    with torch.no_grad():
        lq = net.log_q(th, cfg, sig, chunk=chunk)
        w = torch.exp(lq) * (beta * torch.as_tensor(energies) + lq) / beta
    g = torch.zeros_like(th)
    for b0 in range(0, sig.shape[0], chunk):
        th.grad = None
        s = (w[b0:b0 + chunk] * net.log_q(th, cfg, sig[b0:b0 + chunk], chunk=chunk)).sum()
        s.backward()
        g += th.grad
    return g.detach().numpy()


def Fq_function(theta_t: torch.Tensor, cfg, energies: np.ndarray, beta: float) -> torch.Tensor:
    """F_q(theta) as a differentiable function (for a second route to its gradient)."""
    sig = all_configs(cfg.n_spins)
    lq = net.log_q(theta_t, cfg, sig, chunk=sig.shape[0])
    q = torch.exp(lq)
    return (q * (beta * torch.as_tensor(energies) + lq)).sum() / beta
