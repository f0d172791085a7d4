"""Parity of the local Monte Carlo refinement (checkerboard Metropolis) and of
the self-distillation weights of Eq. (loss2) against the FP64 oracle, through
the C ABI, and of the distillation training step against its composed calls.

Decisions compare a uniform with exp(-beta dE): the kernel in FP32, the oracle
in FP64.  A configuration any of whose decisions came within 1e-5 of the other
outcome (oracle margin) may legitimately diverge from there on; such
configurations are counted and excused, every other one must match exactly
(spins and accepted-flip counts)."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import physics, refine
from tests.gpu_util import FP32, SPLIT, lattice_cfg, say, to_np
from workloads import ea_instance, init_params
from workloads.instances import random_spins

pytestmark = pytest.mark.gpu

TIE = 1e-5


def _compare(inst, spins, beta, sweeps, seed, tag, rows=None):
    g = fv.lmc_graph(inst, sweeps)
    t = torch.as_tensor(spins, device="cuda")
    acc = torch.zeros(spins.shape[0], dtype=torch.int32, device="cuda")
    fv.lmc_refine(g, t, beta, seed, tag, acc)
    torch.cuda.synchronize()
    got, gacc = to_np(t), to_np(acc)
    adj = refine.neighbours(inst.n, inst.edges_i, inst.edges_j, inst.J)
    col = refine.checkerboard_colour(inst.L, inst.dim)
    rows = np.arange(spins.shape[0]) if rows is None else np.asarray(rows)
    bad = 0
    for b in rows:
        ref, racc, marg = refine.metropolis_checkerboard(spins[b:b + 1], adj, col, beta, sweeps, seed, tag, b0=int(b),
                                                          margins=True)
        if marg[0] < TIE:
            bad += 1
            continue
        assert np.array_equal(got[b], ref[0]), f"configuration {b}"
        assert gacc[b] == racc[0]
    return bad, len(rows)


@pytest.mark.parametrize("L,dim,bonds,beta", [(8, 2, "pm1", 0.5), (8, 2, "gauss", 1.3), (4, 3, "gauss", 0.8),
                                              (6, 3, "pm1", 2.0)])
def test_lmc_matches_oracle(L, dim, bonds, beta):
    inst = ea_instance(L, dim, 31, bonds)
    spins = random_spins(48, inst.n, 5)
    say(f"lmc {dim}D L={L} {bonds} beta={beta}")
    bad, n = _compare(inst, spins, beta, 3, seed=(7 << 32) | 99, tag=0x80000003)
    say(f"  {bad} of {n} configurations excused for near-ties")
    assert bad <= 2


def test_lmc_sampled_rows_at_benchmark_size():
    """3D EA L=10, 16384 configurations, 2 sweeps; 12 rows checked against the oracle."""
    inst = ea_instance(10, 3, 1000, "gauss")
    spins = random_spins(16384, inst.n, 9)
    rows = [0, 1, 31, 32, 4095, 8191, 8192, 12000, 16000, 16381, 16382, 16383]
    bad, n = _compare(inst, spins, 1.0, 2, seed=12345, tag=0x80000001, rows=rows)
    assert bad <= 1


def test_lmc_beta_zero_and_zero_sweeps():
    inst = ea_instance(4, 3, 2, "pm1")
    s = random_spins(16, inst.n, 1)
    g = fv.lmc_graph(inst, 1)
    t = torch.as_tensor(s, device="cuda")
    fv.lmc_refine(g, t, 0.0, 1, 1)
    assert np.array_equal(to_np(t), -s)
    g0 = fv.lmc_graph(inst, 0)
    fv.lmc_refine(g0, t, 1.0, 1, 1)
    assert np.array_equal(to_np(t), -s)


@pytest.mark.parametrize("bonds", ["pm1", "gauss"])
def test_distill_weights_match_oracle(bonds):
    inst = ea_instance(6, 2, 4, bonds)
    c = fv.couplings(inst)
    spins = torch.as_tensor(random_spins(257, inst.n, 3), device="cuda")
    E = fv.energy(c, spins)
    lq = torch.as_tensor(np.random.default_rng(2).standard_normal(257).astype(np.float32) * 3 - 20, device="cuda")
    for w in (0.0, 0.5):
        out = to_np(fv.distill_weights(E, lq, 0.9, w)).astype(np.float64)
        ref = refine.distill_weights(to_np(E).astype(np.float64), to_np(lq).astype(np.float64), 0.9, w)
        assert np.max(np.abs(out - ref)) <= 1e-6 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_train_step_distill_equals_composed_calls(prec):
    inst = ea_instance(6, 2, 77, "pm1")
    cfg = lattice_cfg(6, 2, 32, 2, 2)
    B, beta, w, seed, step = 64, 0.8, 0.3, 11, 3
    theta = init_params(cfg, 2, "random")
    m1 = fv.Model(cfg, B, prec, theta)
    m2 = fv.Model(cfg, B, prec, theta)
    c = fv.couplings(inst)
    g = fv.lmc_graph(inst, 2)
    hyper = dict(lr=1e-2, adam_lr=1e-2)
    stats = to_np(m1.train_step_distill(c, g, beta, w, B, seed, step, **hyper))
    spins, lq = m2.sample(B, seed, step)
    E = fv.energy(c, spins)
    st = to_np(fv.free_energy(E, lq, beta, cfg.n_spins))
    fv.lmc_refine(g, spins, beta, seed, 0x80000000 | step)
    E2 = fv.energy(c, spins)
    lq2 = m2.log_prob(spins)
    wts = fv.distill_weights(E2, lq2, beta, w)
    m2.grads.zero_()
    m2.log_prob_backward(spins, wts)
    m2.muon_step(step, **hyper)
    torch.cuda.synchronize()
    assert stats[0] == st[0] and stats[1] == st[1]
    assert np.array_equal(to_np(m1.params), to_np(m2.params))
