"""Shared helpers of the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np
import torch

import paper_2606_22984_amd as fv
from workloads import ModelConfig, init_params, sk_instance, ea_instance
from workloads.instances import lattice_edges

FP32, BF16 = fv.FVAN_FP32, fv.FVAN_BF16
# per-site tolerances of log q and of the sampling decision, by precision
SITE_TOL = {FP32: 1e-4, BF16: 2e-3}
DECISION_TOL = {FP32: 1e-5, BF16: 2e-3}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def masked(cfg: ModelConfig, instance) -> ModelConfig:
    W, P = fv.derive_mask(instance.n, instance.edges_i, instance.edges_j)
    return cfg.with_mask(W, P)


def lattice_cfg(L, D, d, nl, nh, pbc=True):
    ei, ej = lattice_edges(L, D, pbc)
    W, P = fv.derive_mask(L ** D, ei, ej)
    return ModelConfig(L ** D, d, nl, nh).with_mask(W, P)


def make_model(cfg, batch, prec, seed=5, style="random"):
    theta = init_params(cfg, seed, style)
    return fv.Model(cfg, batch, prec, theta), theta


def to_np(t):
    return t.detach().cpu().numpy()
