"""Sampling, backward and the training step of models over 2^D-spin patch
tokens, and of spin models with 32- and 64-wide heads, through the C ABI against
the FP64 oracle (oracle.patch, oracle.network).

Shapes: the 2D EA L=8 lattice in 2x2 patches (16 positions, vocabulary 16) and
the paper's patched 3D EA L=10 model (125 positions of 2x2x2 patches,
vocabulary 256, d_model 128 = 32 token + 96 position dims, 2 heads of width 64,
2 layers; SI, 3D EA settings).

Bars: token decisions as the spin decisions (a token may differ from the
oracle's only where u lies within the precision's decision band of a boundary
of the cumulative distribution between the two tokens), ln q per position as
per site, gradients as the single-spin backward."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import estimator, network as net, patch, philox, physics
from tests.gpu_util import DECISION_TOL, FP32, SITE_TOL, SPLIT, lattice_cfg, make_model, say, to_np
from workloads import ModelConfig, ea_instance, init_params
from workloads.instances import patch_edges, random_spins

pytestmark = pytest.mark.gpu

GRAD_TOL = {FP32: 2e-4, SPLIT: 5e-3}


def _patched_cfg(L, D, d, nl, nh, d_token):
    T, pi, pj = patch_edges(L, D)
    W, P = fv.derive_mask(T, pi, pj)
    return ModelConfig(T, d, nl, nh, d_token=d_token, vocab=2 ** (2 ** D)).with_mask(W, P)


SHAPES = {
    "2d_L8": dict(L=8, D=2, d=32, nl=2, nh=2, d_token=2),
    "3d_L10": dict(L=10, D=3, d=128, nl=2, nh=2, d_token=32),
}


def _check_token_samples(theta, cfg, tok, lq, seed, stream, prec, rows):
    tok = to_np(tok).astype(np.int64)
    lq = to_np(lq).astype(np.float64)
    assert tok.max() < cfg.vocab
    assert np.all(np.isfinite(lq))
    sub = tok[rows]
    th = net.as_theta(theta)
    with torch.no_grad():
        p = torch.softmax(patch.logits_tokens(th, cfg, sub), dim=-1).numpy()       # [R, T, V]
    u = np.concatenate([philox.uniforms(seed, stream, 1, cfg.n_spins, int(b)) for b in rows])   # [R, T]
    R, T, V = p.shape
    ref = patch.categorical_draw(p.reshape(R * T, V), u.reshape(-1)).reshape(R, T)
    # cumulative boundaries C_k = sum_{j >= k} p_j; a differing token is excused
    # only when u lies within the band of a boundary between the two tokens
    C = np.cumsum(p[..., ::-1], axis=-1)[..., ::-1]
    bad = inside = 0
    for r, t in zip(*np.nonzero(ref != sub)):
        lo, hi = sorted((ref[r, t], sub[r, t]))
        gap = np.min(np.abs(u[r, t] - C[r, t, lo + 1:hi + 1]))
        if gap < DECISION_TOL[prec]:
            inside += 1
        else:
            bad += 1
    say(f"token mismatches outside tol: {bad}; inside: {inside} of {sub.size}")
    assert bad == 0
    lref = patch.log_q_tokens(theta, cfg, sub, chunk=8)
    err = np.max(np.abs(lq[rows] - lref)) / cfg.n_spins
    say(f"max per-position |d ln q| {err:.3e}")
    assert err <= SITE_TOL[prec]


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("shape", ["2d_L8", "3d_L10"])
def test_sample_tokens_matches_oracle(prec, shape):
    sh = SHAPES[shape]
    cfg = _patched_cfg(sh["L"], sh["D"], sh["d"], sh["nl"], sh["nh"], sh["d_token"])
    B = 96 if shape == "2d_L8" else 2048
    rows = np.arange(B) if shape == "2d_L8" else np.array([0, 31, 32, 1000, 2047])
    say(f"sample tokens {shape}: T={cfg.n_spins} V={cfg.vocab} W={cfg.window} P={cfg.prefix} "
        f"d_head={cfg.d_head} prec {prec} batch {B}")
    theta = init_params(cfg, 17, "random" if shape == "2d_L8" else "default")
    m = fv.Model(cfg, B, prec, theta)
    tok, lq = m.sample_tokens(B, 41, 3)
    torch.cuda.synchronize()
    m.status()
    _check_token_samples(theta, cfg, tok, lq, 41, 3, prec, rows)
    # the sampled ln q equals the teacher-forced one of the same tokens
    lt = to_np(m.log_prob_tokens(tok)).astype(np.float64)
    assert np.max(np.abs(lt - to_np(lq))) / cfg.n_spins <= SITE_TOL[prec]


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("shape", ["2d_L8", "3d_L10"])
def test_token_backward_matches_oracle(prec, shape):
    sh = SHAPES[shape]
    cfg = _patched_cfg(sh["L"], sh["D"], sh["d"], sh["nl"], sh["nh"], sh["d_token"])
    B = 37 if shape == "2d_L8" else 24
    say(f"token backward {shape}, prec {prec}, batch {B}")
    theta = init_params(cfg, 5, "random")
    m = fv.Model(cfg, B, prec, theta)
    tok = np.random.default_rng(3).integers(0, cfg.vocab, size=(B, cfg.n_spins)).astype(np.uint8)
    w = np.linspace(-1.0, 1.0, B).astype(np.float32)
    m.grads.zero_()
    m.log_prob_tokens_backward(torch.as_tensor(tok, device="cuda"), torch.as_tensor(w, device="cuda"))
    torch.cuda.synchronize()
    m.status()
    g = to_np(m.grads).astype(np.float64)
    gref = patch.grad_surrogate_tokens(theta, cfg, tok, w.astype(np.float64), chunk=8)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    offs, off = {}, 0
    for name, shape in net.layout(cfg):
        offs[name] = off
        off += int(np.prod(shape))
    blocks = {"tok": (0, offs["pos_emb"]), "head": (offs["head.w"], g.size)}
    for name, (a, b) in blocks.items():
        rb = np.linalg.norm(g[a:b] - gref[a:b]) / max(np.linalg.norm(gref[a:b]), 1e-30)
        say(f"  {name} block rel. error {rb:.2e}")
        assert rb <= GRAD_TOL[prec]
    say(f"  gradient rel. error {rel:.2e}")
    assert rel <= GRAD_TOL[prec]


def test_tokens_to_spins_is_the_patch_map():
    for L, D in ((8, 2), (10, 3), (6, 1)):
        sites = torch.as_tensor(fv.patch_sites(L, D), device="cuda")
        T, bits = sites.shape
        tok = np.random.default_rng(L).integers(0, 2 ** bits, size=(33, T)).astype(np.uint8)
        got = to_np(fv.tokens_to_spins(sites, torch.as_tensor(tok, device="cuda")))
        assert np.array_equal(got, patch.tokens_to_spins(tok, L, D))


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_train_step_tokens(prec):
    """One patched training step equals the composed calls bit for bit, and its
    F_q statistics match the oracle's re-evaluation of the step's samples."""
    L, D = 8, 2
    cfg = _patched_cfg(L, D, 32, 2, 2, 2)
    inst = ea_instance(L, D, 4, "pm1")
    coup = fv.couplings(inst)
    sites = torch.as_tensor(fv.patch_sites(L, D), device="cuda")
    B, beta, seed, step = 256, 1.3, 9, 4
    theta = init_params(cfg, 8, "random")
    a = fv.Model(cfg, B, prec, theta)
    b = fv.Model(cfg, B, prec, theta)
    hyper = dict(lr=2e-2, adam_lr=1e-2)
    st = to_np(a.train_step_tokens(coup, sites, beta, B, seed, step, **hyper))
    a.status()
    # composed: sample -> spins -> energy -> F_q -> weights -> backward -> Muon
    tok, lq = b.sample_tokens(B, seed, step)
    spins = fv.tokens_to_spins(sites, tok)
    E = coup.empty_energy(B)
    fv.energy(coup, spins, E)
    st2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    fv.free_energy(E, lq, beta, L ** D, st2)
    w = torch.empty(B, dtype=torch.float32, device="cuda")
    fv.reinforce_weights(E, lq, beta, w)
    b.log_prob_tokens_backward(tok, w)
    b.muon_step(step, **hyper)
    torch.cuda.synchronize()
    assert np.array_equal(st[:2], to_np(st2))
    assert torch.equal(a.params, b.params)
    # the oracle on the step's own samples, at the parameters they were drawn with
    sp = to_np(spins)
    E_ref = physics.energy_edges(sp, inst.edges_i, inst.edges_j, inst.J)
    lq_ref = patch.log_q_tokens(theta, cfg, to_np(tok).astype(np.int64))
    f_ref, _ = estimator.free_energy_stats(E_ref, lq_ref, beta, L ** D)
    say(f"patched step, prec {prec}: F_q/N {st[0]:.6f} vs oracle {f_ref:.6f}")
    assert abs(st[0] - f_ref) <= 1e-4
    assert np.array_equal(to_np(E).astype(np.float64), E_ref)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("d_head", [32, 64])
def test_spin_model_with_wide_heads(prec, d_head):
    """Sampling, teacher-forced ln q and the backward of a spin model whose heads
    are 32 or 64 wide (the FP32 attention kernels and the wider decode heads)."""
    cfg = lattice_cfg(6, 2, 64, 2, 64 // d_head)
    B = 70
    say(f"wide heads: d_head {d_head}, prec {prec}")
    m, theta = make_model(cfg, B, prec, seed=12)
    spins, lq = m.sample(B, seed=6, stream_id=2)
    torch.cuda.synchronize()
    sp = to_np(spins)
    th = net.as_theta(theta)
    pp = net.cond_plus(th, cfg, sp, chunk=16).numpy()
    u = philox.uniforms(6, 2, B, cfg.n_spins)
    wrong = (u < pp) != (sp > 0)
    assert int((wrong & (np.abs(u - pp) >= DECISION_TOL[prec])).sum()) == 0
    ref = net.log_q(th, cfg, sp, chunk=16).numpy()
    assert np.max(np.abs(to_np(lq) - ref)) / cfg.n_spins <= SITE_TOL[prec]
    s2 = random_spins(B, cfg.n_spins, 4)
    lt = to_np(m.log_prob(torch.as_tensor(s2, device="cuda"))).astype(np.float64)
    assert np.max(np.abs(lt - net.log_q(th, cfg, s2, chunk=16).numpy())) / cfg.n_spins <= SITE_TOL[prec]
    w = torch.linspace(-1.0, 1.0, B, device="cuda")
    m.grads.zero_()
    m.log_prob_backward(torch.as_tensor(s2, device="cuda"), w)
    torch.cuda.synchronize()
    g = to_np(m.grads).astype(np.float64)
    gref = estimator.grad_surrogate(theta, cfg, s2, to_np(w).astype(np.float64))
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say(f"  gradient rel. error {rel:.2e}")
    assert rel <= GRAD_TOL[prec]
