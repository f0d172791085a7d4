"""Degenerate cases of the method on the HIP path against the oracle: the
zero-layer model (the transformer reduces to a position-wise logistic model of
the previous spin, with a closed form the oracle is pinned to), through
sampling, teacher-forced log q, the backward and one Muon step."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import estimator, muon, network as net
from tests.gpu_util import ALL_PRECISIONS, FP32, SITE_TOL, SPLIT, make_model, say, to_np
from tests.test_gpu_sample import _check_samples
from workloads import ModelConfig
from workloads.instances import random_spins

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ALL_PRECISIONS)
def test_zero_layer_model(prec):
    cfg = ModelConfig(12, 32, 0, 2).full_causal()
    B = 96
    m, theta = make_model(cfg, B, prec, seed=13)
    say(f"zero layers, prec {prec}")
    spins, lq = m.sample(B, seed=4, stream_id=9)
    torch.cuda.synchronize()
    _check_samples(theta, cfg, spins, lq, 4, 9, prec)
    s = torch.as_tensor(random_spins(B, cfg.n_spins, 2), device="cuda")
    lt = to_np(m.log_prob(s)).astype(np.float64)
    ref = net.log_q(net.as_theta(theta), cfg, to_np(s)).numpy()
    assert np.max(np.abs(lt - ref)) / cfg.n_spins <= SITE_TOL[prec]
    w = torch.linspace(-1.0, 1.0, B, device="cuda")
    m.grads.zero_()
    m.log_prob_backward(s, w)
    torch.cuda.synchronize()
    g = to_np(m.grads).astype(np.float64)
    gref = estimator.grad_surrogate(theta, cfg, to_np(s), to_np(w).astype(np.float64))
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say(f"  gradient rel. error {rel:.2e}")
    assert rel <= {fv.FVAN_FP32: 2e-4, fv.FVAN_BF16_SPLIT: 5e-3}[prec]
    if prec == FP32:
        n = g.size
        new, _, _ = muon.muon_update(theta.astype(np.float64), g, np.zeros(n), np.zeros(n), 1, cfg, 1e-2,
                                     adam_lr=1e-3)
        m.muon_step(1, lr=1e-2, adam_lr=1e-3)
        torch.cuda.synchronize()
        assert np.max(np.abs(to_np(m.params) - new)) <= 1e-6


def test_binding_refuses_malformed_spin_tensors():
    """The C entry points read batch x n int8 spins from a pointer; the binding
    refuses tensors of another width or dtype, or too few rows, before any launch."""
    from workloads import ModelConfig, init_params
    cfg = ModelConfig(16, 32, 2, 2).with_mask(4, 4)
    m = fv.Model(cfg, 8, fv.FVAN_FP32, init_params(cfg, 1, "random"))
    good = torch.ones(8, 16, dtype=torch.int8, device="cuda")
    for bad in (torch.ones(8, 15, dtype=torch.int8, device="cuda"), torch.ones(8, 16, dtype=torch.int32, device="cuda"),
                torch.ones(16, dtype=torch.int8, device="cuda")):
        with pytest.raises(ValueError):
            m.log_prob(bad)
        with pytest.raises(ValueError):
            m.log_prob_backward(bad, torch.zeros(8, device="cuda"))
    with pytest.raises(ValueError):
        m.log_prob_backward(good, torch.zeros(7, device="cuda"))
    with pytest.raises(ValueError):
        m.sample(8, 1, 1, spins=torch.empty(4, 16, dtype=torch.int8, device="cuda"))
    with pytest.raises(ValueError):
        m.log_prob(good, log_q=torch.empty(8, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
