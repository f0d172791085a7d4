"""Conventions of the C ABI on the GPU: every workspace is allocated at create
time (no later call allocates device memory), a model created without a
workspace refuses the calls that need it, and non-finite results are reported
as FVAN_ENONFINITE by the next synchronising call."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from tests.gpu_util import FP32, SPLIT, lattice_cfg, make_model, say
from workloads import ea_instance, init_params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_first_teacher_forced_calls_allocate_nothing(prec):
    cfg = lattice_cfg(16, 2, 64, 4, 4)
    B = 512
    theta = init_params(cfg, 3, "random")
    # load every kernel's code object first, on a throwaway model of the same kind
    warm = fv.Model(cfg, 40, prec, theta)
    s, _ = warm.sample(40, 1, 1)
    warm.log_prob(s)
    warm.log_prob_backward(s, torch.ones(40, device="cuda"))
    torch.cuda.synchronize()
    m = fv.Model(cfg, B, prec, theta)
    spins, _ = m.sample(B, 5, 2)
    lq = torch.empty(B, dtype=torch.float32, device="cuda")
    w = torch.linspace(-1.0, 1.0, B, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    m.log_prob(spins, lq)
    m.log_prob_backward(spins, w)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say(f"prec {prec}: free device memory {free0} -> {free1}")
    assert free1 == free0


def test_workspaces_select_the_calls():
    cfg = lattice_cfg(6, 2, 32, 2, 2)
    theta = init_params(cfg, 2, "random")
    ms = fv.Model(cfg, 64, FP32, theta, workspaces=fv.WS_SAMPLER)
    spins, _ = ms.sample(64, 1, 1)
    with pytest.raises(fv.FvanError, match="EUNSUPPORTED"):
        ms.log_prob(spins)
    with pytest.raises(fv.FvanError, match="EUNSUPPORTED"):
        ms.log_prob_backward(spins, torch.ones(64, device="cuda"))
    with pytest.raises(fv.FvanError, match="EUNSUPPORTED"):
        ms.muon_step(1)
    mt = fv.Model(cfg, 64, FP32, theta, workspaces=fv.WS_TEACHER)
    lq = mt.log_prob(spins)
    with pytest.raises(fv.FvanError, match="EUNSUPPORTED"):
        mt.sample(64, 1, 1)
    inst = ea_instance(6, 2, 7, "pm1")
    with pytest.raises(fv.FvanError, match="EUNSUPPORTED"):
        mt.train_step_muon(fv.couplings(inst), 1.0, 64, 1, 1)
    torch.cuda.synchronize()
    assert torch.isfinite(lq).all()
    with pytest.raises(fv.FvanError, match="EINVAL"):
        fv.Model(cfg, 64, 1, theta)          # plain-BF16 operands are not a mode of this library


def test_nonfinite_parameters_are_reported():
    cfg = lattice_cfg(6, 2, 32, 2, 2)
    inst = ea_instance(6, 2, 8, "pm1")
    c = fv.couplings(inst)
    m, theta = make_model(cfg, 64, SPLIT, seed=4)
    m.train_step_muon(c, 1.0, 64, 3, 1)
    m.status()                                 # finite so far
    m.train_step_muon(c, 1.0, 64, 3, 2)        # waits for step 1: finite, so it proceeds
    bad = theta.copy()
    bad[-5] = np.nan                           # a head weight
    m.set_params(bad)
    say("NaN written into the head weights")
    m.train_step_muon(c, 1.0, 64, 3, 3)        # enqueued; its check runs on the device
    with pytest.raises(fv.FvanError, match="ENONFINITE"):
        m.train_step_muon(c, 1.0, 64, 3, 4)    # reports step 3 and enqueues nothing
    m.status()                                 # that report cleared the flag
    # a sampling call alone: reported by the synchronising status call.  (An
    # infinite head weight would not do: it saturates p to 0 or 1 and the drawn
    # spin's log-probability is then exactly 0, a finite ln q.)
    m2, th2 = make_model(cfg, 32, FP32, seed=5)
    th2 = th2.copy()
    th2[-5] = np.nan
    m2.set_params(th2)
    m2.sample(32, 1, 1)
    with pytest.raises(fv.FvanError, match="ENONFINITE"):
        m2.status()
    m2.status()
