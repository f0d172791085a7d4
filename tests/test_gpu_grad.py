"""Parity of the teacher-forced log q, the hand-written backward and the training
step (HIP path) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import estimator, exact, network as net, physics
from tests.gpu_util import ALL_PRECISIONS, FP32, SITE_TOL, SPLIT, lattice_cfg, make_model, say, to_np
from workloads import ModelConfig, ea_instance, init_params, sk_instance
from workloads.instances import random_spins

pytestmark = pytest.mark.gpu

# relative L2 error of a gradient vector, by precision
GRAD_TOL = {FP32: 2e-4, SPLIT: 5e-3}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("prec", ALL_PRECISIONS)
def test_log_prob_normalised_by_enumeration_sk16(prec):
    """All 2^16 configurations through the teacher-forced GPU pass: sum q = 1."""
    cfg = ModelConfig(16, 32, 2, 2).full_causal()
    sig = torch.as_tensor(__import__("oracle").physics.all_configs(16), device="cuda")
    m, theta = make_model(cfg, sig.shape[0], prec, seed=3)
    lq = to_np(m.log_prob(sig)).astype(np.float64)
    total = np.exp(lq).sum()
    say(f"prec {prec}: sum q = {total:.8f}")
    assert abs(total - 1.0) <= {FP32: 1e-5, SPLIT: 1e-3}[prec]
    ref = net.log_q(net.as_theta(theta), cfg, to_np(sig)[::257], chunk=256).numpy()
    assert np.max(np.abs(lq[::257] - ref)) / 16 <= SITE_TOL[prec]


@pytest.mark.parametrize("prec", ALL_PRECISIONS)
@pytest.mark.parametrize("shape", ["band", "ea2d", "sk512"])
def test_log_prob_matches_oracle(prec, shape):
    if shape == "band":
        cfg, B, rows = ModelConfig(40, 64, 3, 4).with_mask(6, 5), 37, None
    elif shape == "ea2d":
        cfg, B, rows = lattice_cfg(16, 2, 64, 4, 4), 24, None
    else:
        cfg, B, rows = ModelConfig(512, 128, 6, 8).full_causal(), 6, [0, 5]
    m, theta = make_model(cfg, B, prec, seed=4)
    spins = torch.as_tensor(random_spins(B, cfg.n_spins, 7), device="cuda")
    lq = to_np(m.log_prob(spins)).astype(np.float64)
    idx = np.arange(B) if rows is None else np.asarray(rows)
    ref = net.log_q(net.as_theta(theta), cfg, to_np(spins)[idx], chunk=8).numpy()
    err = np.max(np.abs(lq[idx] - ref)) / cfg.n_spins
    say(f"{shape} prec {prec}: max per-site |d ln q| = {err:.3e}")
    assert err <= SITE_TOL[prec]


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_log_prob_multi_chunk_ea3d(prec):
    """3D shape: more samples than one chunk of rows (ragged last chunk)."""
    cfg = lattice_cfg(10, 3, 128, 8, 8)
    B = 4200
    m, theta = make_model(cfg, B, prec, seed=21, style="default")
    spins, lq_s = m.sample(B, 3, 3)
    lq_t = m.log_prob(spins)
    torch.cuda.synchronize()
    d = to_np(lq_t - lq_s).astype(np.float64)
    say(f"prec {prec}: sampled vs teacher-forced per-site max {np.abs(d).max() / cfg.n_spins:.3e}")
    assert np.abs(d).max() / cfg.n_spins <= SITE_TOL[prec]
    rows = [0, 2096, 2097, 4199]
    ref = net.log_q(net.as_theta(theta), cfg, to_np(spins)[rows], chunk=2).numpy()
    assert np.max(np.abs(to_np(lq_t)[rows] - ref)) / cfg.n_spins <= SITE_TOL[prec]


@pytest.mark.parametrize("prec", ALL_PRECISIONS)
@pytest.mark.parametrize("shape", ["band", "full"])
def test_backward_matches_oracle_gradient(prec, shape):
    if shape == "band":
        cfg = ModelConfig(70, 64, 2, 4).with_mask(9, 7)
    else:
        cfg = ModelConfig(24, 32, 3, 2).full_causal()
    B = 21
    m, theta = make_model(cfg, B, prec, seed=6)
    spins_np = random_spins(B, cfg.n_spins, 2)
    c = np.random.default_rng(3).standard_normal(B).astype(np.float32)
    spins = torch.as_tensor(spins_np, device="cuda")
    m.grads.zero_()
    m.log_prob_backward(spins, torch.as_tensor(c, device="cuda"))
    g = to_np(m.grads).astype(np.float64)
    ref = estimator.grad_surrogate(theta, cfg, spins_np, c.astype(np.float64))
    rel = _rel(g, ref)
    say(f"{shape} prec {prec}: relative gradient error {rel:.3e}")
    assert rel <= GRAD_TOL[prec]
    # accumulation semantics: a second call adds the same gradient again
    m.log_prob_backward(spins, torch.as_tensor(c, device="cuda"))
    g2 = to_np(m.grads).astype(np.float64)
    assert _rel(g2, 2 * g) <= 1e-5


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_backward_sk512_sampled_coordinates(prec):
    """SK N=512 shape (d=128, 6 layers, 8 heads): GPU gradient vs oracle reverse mode on 64
    random coordinates, 8 samples with baseline-subtracted REINFORCE weights."""
    cfg = ModelConfig(512, 128, 6, 8).full_causal()
    inst = sk_instance(512, 3000)
    B = 8
    m, theta = make_model(cfg, B, prec, seed=31, style="default")
    spins, lq = m.sample(B, 4, 1)
    c = fv.couplings(inst)
    E = fv.energy(c, spins)
    w = fv.reinforce_weights(E, lq, 1.5)
    m.grads.zero_()
    m.log_prob_backward(spins, w)
    g = to_np(m.grads).astype(np.float64)
    ref = estimator.grad_surrogate(theta, cfg, to_np(spins), to_np(w).astype(np.float64), chunk=2)
    idx = np.random.default_rng(0).choice(g.shape[0], 64, replace=False)
    scale = np.abs(ref).max()
    err = np.max(np.abs(g[idx] - ref[idx])) / scale
    say(f"prec {prec}: max |dg| / max|g| on 64 coordinates = {err:.3e}; full rel {_rel(g, ref):.3e}")
    assert err <= {FP32: 1e-4, SPLIT: 2e-3}[prec]
    assert _rel(g, ref) <= GRAD_TOL[prec]


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_backward_full_batch_ea3d_sampled_rows(prec):
    """The benchmark's launch: 3D L=10 model (d=128, 8 layers, 8 heads), 16384
    samples, so the backward runs its row chunks (2097 samples each, a ragged last
    one).  Weights are zero except on four samples (both sides of the first chunk
    boundary and the two batch ends); zero-weight rows add exact zeros, so the GPU
    gradient is the oracle's gradient of those four samples."""
    cfg = lattice_cfg(10, 3, 128, 8, 8)
    B = 16384
    m, theta = make_model(cfg, B, prec, seed=21, style="default")
    spins_np = random_spins(B, cfg.n_spins, 12)
    rows = [0, 2096, 2097, B - 1]
    c = np.zeros(B, dtype=np.float32)
    c[rows] = [0.7, -1.3, 0.4, 1.1]
    say(f"ea3d full-batch backward, prec {prec}")
    m.grads.zero_()
    m.log_prob_backward(torch.as_tensor(spins_np, device="cuda"), torch.as_tensor(c, device="cuda"))
    g = to_np(m.grads).astype(np.float64)
    ref = estimator.grad_surrogate(theta, cfg, spins_np[rows], c[rows].astype(np.float64), chunk=1)
    rel = _rel(g, ref)
    say(f"  relative gradient error {rel:.3e}")
    assert rel <= GRAD_TOL[prec]


def test_autograd_function_matches_direct_backward():
    cfg = ModelConfig(30, 32, 2, 2).with_mask(4, 2)
    m, theta = make_model(cfg, 12, FP32, seed=8)
    spins = torch.as_tensor(random_spins(12, 30, 1), device="cuda")
    params = m.params.clone().requires_grad_(True)
    lq = fv.LogProb.apply(params, m, spins)
    w = torch.linspace(-1, 1, 12, device="cuda")
    (lq * w).sum().backward()
    m.grads.zero_()
    m.log_prob_backward(spins, w.contiguous())
    assert torch.allclose(params.grad, m.grads, rtol=0, atol=0)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_train_step_equals_composed_calls_and_oracle_adam(prec):
    """fvan_train_step == sample -> energy -> weights -> backward -> Adam done call by call;
    the Adam update matches the oracle's on the same gradient."""
    inst = ea_instance(6, 2, 77, "pm1")
    cfg = lattice_cfg(6, 2, 32, 2, 2)
    B, beta, seed, step = 64, 0.8, 11, 1
    theta = init_params(cfg, 2, "random")
    m1 = fv.Model(cfg, B, prec, theta)
    m2 = fv.Model(cfg, B, prec, theta)
    c = fv.couplings(inst)
    stats = to_np(m1.train_step(c, beta, B, seed, step, lr=1e-2))
    spins, lq = m2.sample(B, seed, step)
    E = fv.energy(c, spins)
    st = to_np(fv.free_energy(E, lq, beta, cfg.n_spins))
    w = fv.reinforce_weights(E, lq, beta)
    m2.grads.zero_()
    m2.log_prob_backward(spins, w)
    g = to_np(m2.grads).astype(np.float64)
    m2.adam_step(step, lr=1e-2)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(m1.params), to_np(m2.params))
    assert stats[0] == st[0] and stats[1] == st[1]
    assert abs(stats[2] - to_np(E).astype(np.float64).mean() / cfg.n_spins) < 1e-12
    assert abs(stats[3] - np.linalg.norm(g)) <= 1e-5 * np.linalg.norm(g)
    new, _, _ = estimator.adam_update(theta.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), step, 1e-2)
    assert np.max(np.abs(to_np(m2.params) - new)) <= 1e-6


def test_training_lowers_free_energy_sk16():
    """A few Adam steps of the full GPU step on SK N=16 lower F_q toward the exact F, and F_q >= F."""
    inst = sk_instance(16, 1000)
    cfg = ModelConfig(16, 32, 2, 2).full_causal()
    beta = 1.0
    m, theta = make_model(cfg, 1024, FP32, seed=7, style="default")
    c = fv.couplings(inst)
    E_all = physics.energy_dense(physics.all_configs(16), inst.dense)
    Fq0, F, _ = exact.exact_free_energies(to_np(m.params), cfg, E_all, beta)
    for step in range(1, 61):
        m.train_step(c, beta, 1024, 5, step, lr=3e-3)
    torch.cuda.synchronize()
    Fq1, _, s = exact.exact_free_energies(to_np(m.params), cfg, E_all, beta)
    say(f"F = {F / 16:.5f}; F_q before {Fq0 / 16:.5f}, after {Fq1 / 16:.5f}")
    assert abs(s - 1) < 1e-9
    assert Fq1 >= F - 1e-9
    assert Fq1 < Fq0 - 0.2 * (Fq0 - F)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_backward_on_a_caller_stream_matches_default_stream(prec):
    """The backward forks its weight gradients onto a stream of the model and joins
    it back: on a non-default caller stream, with calls queued back to back and a
    gradient reset between them on that stream, the result is bitwise the
    default-stream one (the reductions have a fixed order)."""
    cfg = ModelConfig(40, 64, 3, 4).with_mask(6, 3)
    m, theta = make_model(cfg, 24, prec, seed=21)
    spins = torch.as_tensor(random_spins(24, 40, 5), device="cuda")
    w = torch.linspace(-1, 1, 24, device="cuda")
    m.grads.zero_()
    m.log_prob_backward(spins, w)
    torch.cuda.synchronize()
    ref = m.grads.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            m.grads.zero_()
            m.log_prob_backward(spins, w)
        out = m.grads.clone()
    torch.cuda.synchronize()
    say(f"caller-stream backward, precision {prec}")
    assert torch.equal(out, ref)
