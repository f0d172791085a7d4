"""Parity of the Muon update (Newton-Schulz orthogonalisation on FP32 MFMA,
momentum, scaled step with decoupled weight decay, Adam on the non-matrix
parameters) against the FP64 oracle, through the C ABI.

Tolerance: the Newton-Schulz output is compared element by element with
|O_gpu - O_oracle| <= 5e-5 max|O_oracle|.  The same iteration run in float32
with numpy stays within 5.2e-6 max|O| on every shape below (the Gram and
polynomial products round once per product at FP32; five iterations of the
quintic leave that at the 1e-6 level); the bar is ten times that."""
import math

import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import exact, muon, network as net, physics, estimator
from tests.gpu_util import FP32, SPLIT, lattice_cfg, make_model, say, to_np
from workloads import ModelConfig, ea_instance, init_params, sk_instance

pytestmark = pytest.mark.gpu

NS_TOL = 5e-5
SHAPES = [(128, 512), (512, 128), (384, 128), (128, 384), (40, 100), (100, 40), (1, 7), (7, 1), (16, 16),
          (128, 128), (64, 2000), (33, 129), (129, 33), (5, 3)]


def _gauss(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)


@pytest.mark.parametrize("shape", SHAPES)
def test_newton_schulz_matches_oracle(shape):
    M = _gauss(shape, shape[0] * 7919 + shape[1])
    say(f"newton_schulz {shape}")
    out = to_np(fv.newton_schulz(torch.as_tensor(M, device="cuda")))
    ref = muon.newton_schulz(M.astype(np.float64))
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    say(f"  max |dO| / max|O| = {err:.2e}")
    assert err <= NS_TOL


@pytest.mark.parametrize("steps", [0, 1, 3, 16])
def test_newton_schulz_step_counts(steps):
    M = _gauss((48, 80), 11 + steps)
    out = to_np(fv.newton_schulz(torch.as_tensor(M, device="cuda"), steps=steps, eps=1e-3))
    ref = muon.newton_schulz(M.astype(np.float64), steps, 1e-3)
    assert np.max(np.abs(out - ref)) <= NS_TOL * np.max(np.abs(ref))


def test_newton_schulz_in_place_and_known_svd():
    """In place equals out of place bitwise, and both follow the singular-value
    closed form U diag(p^5(s / ||s||)) V^T of a matrix built from its SVD."""
    rng = np.random.default_rng(3)
    r, c = 96, 200
    U = np.linalg.qr(rng.standard_normal((r, r)))[0]
    V = np.linalg.qr(rng.standard_normal((c, r)))[0]
    s = np.linspace(0.2, 5.0, r)
    M = ((U * s) @ V.T).astype(np.float32)
    x = s / np.linalg.norm(s)
    for _ in range(5):
        x = 3.4445 * x - 4.7750 * x ** 3 + 2.0315 * x ** 5
    want = (U * x) @ V.T
    t = torch.as_tensor(M, device="cuda")
    out = to_np(fv.newton_schulz(t))
    fv.newton_schulz(t, out=t)
    assert np.array_equal(to_np(t), out)
    assert np.max(np.abs(out - want)) <= NS_TOL * np.max(np.abs(want))


def test_newton_schulz_zero_matrix_stays_zero():
    out = to_np(fv.newton_schulz(torch.zeros(32, 64, device="cuda")))
    assert not np.any(out)


def _tol_w(theta, lr, scale_max, O_max=1.0):
    return lr * scale_max * NS_TOL * O_max + 4e-7 * max(1.0, float(np.max(np.abs(theta))))


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("shape", ["d32", "d128"])
def test_muon_step_matches_oracle(prec, shape):
    """Two Muon steps (momentum carried) on random gradients; every parameter
    against the oracle, gradients cleared, packed weights refreshed."""
    cfg = ModelConfig(30, 32, 2, 2).with_mask(4, 2) if shape == "d32" else ModelConfig(20, 128, 2, 8).full_causal()
    m, theta = make_model(cfg, 4, prec, seed=9)
    n = theta.size
    rng = np.random.default_rng(21)
    hyper = dict(lr=2e-2, momentum=0.9, weight_decay=0.05, rms_scale=0.2, ns_eps=1e-7, ns_steps=5, adam_lr=1e-2,
                 adam_weight_decay=0.01)
    ref_t, ref_m, ref_v = theta.astype(np.float64), np.zeros(n), np.zeros(n)
    scale_max = 0.2 * math.sqrt(4 * cfg.d_model)
    for step in (1, 2):
        g = (rng.standard_normal(n) * 1e-2).astype(np.float32)
        m.grads.copy_(torch.as_tensor(g, device="cuda"))
        say(f"muon step {step}, {shape}, prec {prec}")
        m.muon_step(step, **hyper)
        torch.cuda.synchronize()
        ref_t, ref_m, ref_v = muon.muon_update(ref_t, g.astype(np.float64), ref_m, ref_v, step, cfg, **hyper)
        got = to_np(m.params).astype(np.float64)
        mask = muon.muon_entries(cfg)
        err_mat = np.max(np.abs(got[mask] - ref_t[mask]))
        err_rest = np.max(np.abs(got[~mask] - ref_t[~mask]))
        say(f"  max |dW| matrices {err_mat:.2e}, others {err_rest:.2e}")
        assert err_mat <= _tol_w(ref_t, hyper["lr"], scale_max)
        assert err_rest <= 1e-6
        assert not torch.any(m.grads)
    # the packed copies follow the new parameters: log q equals a fresh model's
    spins = torch.as_tensor(np.where(rng.random((4, cfg.n_spins)) < 0.5, -1, 1).astype(np.int8), device="cuda")
    m2 = fv.Model(cfg, 4, prec, to_np(m.params))
    assert torch.equal(m.log_prob(spins), m2.log_prob(spins))


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_train_step_muon_equals_composed_calls(prec):
    """fvan_train_step_muon == sample -> energy -> weights -> backward -> Muon,
    call by call, bitwise; same statistics as the Adam train step."""
    inst = ea_instance(6, 2, 77, "pm1")
    cfg = lattice_cfg(6, 2, 32, 2, 2)
    B, beta, seed, step = 64, 0.8, 11, 1
    theta = init_params(cfg, 2, "random")
    m1 = fv.Model(cfg, B, prec, theta)
    m2 = fv.Model(cfg, B, prec, theta)
    c = fv.couplings(inst)
    hyper = dict(lr=1e-2, adam_lr=1e-2)
    stats = to_np(m1.train_step_muon(c, beta, B, seed, step, **hyper))
    spins, lq = m2.sample(B, seed, step)
    E = fv.energy(c, spins)
    st = to_np(fv.free_energy(E, lq, beta, cfg.n_spins))
    w = fv.reinforce_weights(E, lq, beta)
    m2.grads.zero_()
    m2.log_prob_backward(spins, w)
    m2.muon_step(step, **hyper)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(m1.params), to_np(m2.params))
    assert stats[0] == st[0] and stats[1] == st[1]


def test_muon_training_lowers_free_energy_sk12():
    """Muon steps of the full GPU training step on SK N=12 lower F_q toward the
    exact F (enumerated), and F_q >= F throughout."""
    inst = sk_instance(12, 1000)
    cfg = ModelConfig(12, 32, 2, 2).full_causal()
    beta = 1.0
    m, theta = make_model(cfg, 1024, FP32, seed=7, style="default")
    c = fv.couplings(inst)
    E_all = physics.energy_dense(physics.all_configs(12), inst.dense)
    Fq0, F, _ = exact.exact_free_energies(to_np(m.params), cfg, E_all, beta)
    for step in range(1, 61):
        m.train_step_muon(c, beta, 1024, 5, step, lr=1e-2, adam_lr=3e-3)
    torch.cuda.synchronize()
    Fq1, _, s = exact.exact_free_energies(to_np(m.params), cfg, E_all, beta)
    say(f"F = {F / 12:.5f}; F_q before {Fq0 / 12:.5f}, after {Fq1 / 12:.5f}")
    assert abs(s - 1) < 1e-9
    assert Fq1 >= F - 1e-9
    assert Fq1 < Fq0 - 0.2 * (Fq0 - F)


def test_muon_rejects_bad_hyper_parameters():
    cfg = ModelConfig(30, 32, 2, 2).with_mask(4, 2)
    m, theta = make_model(cfg, 4, FP32, seed=1)
    for bad in (dict(momentum=1.0), dict(ns_steps=17), dict(ns_eps=0.0), dict(lr=-1.0), dict(adam_beta1=1.0),
                dict(rms_scale=float("nan"))):
        with pytest.raises(fv.FvanError):
            m.muon_step(1, **bad)
    assert np.array_equal(to_np(m.params), theta)
