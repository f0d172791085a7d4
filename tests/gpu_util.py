"""Shared helpers of the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np
import torch

import paper_2606_22984_amd as fv
from workloads import ModelConfig, init_params, sk_instance, ea_instance
from workloads.instances import lattice_edges

FP32, SPLIT = fv.FVAN_FP32, fv.FVAN_BF16_SPLIT
ALL_PRECISIONS = (FP32, SPLIT)
# Tolerances by precision, the bars of the method's parity spec: per-site log q
# (|d ln q_b| / N: 1e-4 in FP32, 2e-3 in the BF16 path) and the band of |u - p|
# inside which a sampling decision may differ from the oracle's (1e-5 in FP32,
# 2e-3 in the BF16 path).
SITE_TOL = {FP32: 1e-4, SPLIT: 2e-3}
DECISION_TOL = {FP32: 1e-5, SPLIT: 2e-3}


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
