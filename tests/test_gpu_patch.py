"""Teacher-forced ln q of models over 2^D-spin patch tokens (vocabulary 16 in 2D,
256 in 3D) through the C ABI, against the FP64 oracle (oracle.patch).

Tolerance: |d ln q| / T per sample, T = number of token positions, the same
per-position bars as the single-spin teacher-forced pass."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import patch
from tests.gpu_util import FP32, SITE_TOL, SPLIT, say, to_np
from workloads import ModelConfig, init_params
from workloads.instances import lattice_edges, random_spins

pytestmark = pytest.mark.gpu


def _patched_cfg(L, D, d, nl, nh):
    """Model over the (L/2)^D patches of a periodic L^D lattice; mask derived from
    the patch graph (two patches interact if any of their sites do)."""
    sites = patch.patch_sites(L, D)
    owner = np.empty(L ** D, dtype=np.int64)
    owner[sites.reshape(-1)] = np.repeat(np.arange(sites.shape[0]), sites.shape[1])
    ei, ej = lattice_edges(L, D, True)
    pi, pj = owner[np.asarray(ei)], owner[np.asarray(ej)]
    keep = pi != pj
    pairs = np.unique(np.sort(np.stack([pi[keep], pj[keep]], 1), axis=1), axis=0)
    T = sites.shape[0]
    W, P = fv.derive_mask(T, pairs[:, 0].astype(np.int32), pairs[:, 1].astype(np.int32))
    return ModelConfig(T, d, nl, nh, vocab=2 ** (2 ** D)).with_mask(W, P)


def _tokens(batch, T, V, seed):
    return np.random.default_rng(seed).integers(0, V, size=(batch, T)).astype(np.uint8)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("shape", ["2d", "3d"])
def test_log_prob_tokens_matches_oracle(prec, shape):
    if shape == "2d":
        cfg, B, rows = _patched_cfg(8, 2, 32, 2, 2), 37, None
    else:
        cfg, B, rows = _patched_cfg(10, 3, 128, 8, 8), 16384, [0, 8191, 16383]
    say(f"patched {shape}: T={cfg.n_spins}, V={cfg.vocab}, mask W={cfg.window} P={cfg.prefix}, prec {prec}")
    theta = init_params(cfg, 13, "random" if shape == "2d" else "default")
    m = fv.Model(cfg, B, prec, theta)
    tok = _tokens(B, cfg.n_spins, cfg.vocab, 5)
    lq = to_np(m.log_prob_tokens(torch.as_tensor(tok, device="cuda"))).astype(np.float64)
    assert np.all(np.isfinite(lq))
    idx = np.arange(B) if rows is None else np.asarray(rows)
    ref = patch.log_q_tokens(theta, cfg, tok[idx], chunk=4)
    err = np.max(np.abs(lq[idx] - ref)) / cfg.n_spins
    say(f"  max |d ln q| / T = {err:.3e}")
    assert err <= SITE_TOL[prec]


def test_log_prob_tokens_normalised_by_enumeration():
    """4x4 lattice in 2x2 patches: the 16^4 token sequences are every spin state
    once; the GPU's q sums to 1."""
    cfg = ModelConfig(4, 32, 2, 2, vocab=16).with_mask(1, 1)
    theta = init_params(cfg, 3, "random")
    allseq = np.stack(np.meshgrid(*[np.arange(16)] * 4, indexing="ij"), -1).reshape(-1, 4).astype(np.uint8)
    m = fv.Model(cfg, allseq.shape[0], FP32, theta)
    lq = to_np(m.log_prob_tokens(torch.as_tensor(allseq, device="cuda"))).astype(np.float64)
    total = np.exp(lq).sum()
    say(f"sum q = {total:.8f}")
    assert abs(total - 1.0) < 1e-4


def test_vocab_two_tokens_equal_the_spin_pass():
    cfg = ModelConfig(30, 32, 2, 2).with_mask(4, 2)
    theta = init_params(cfg, 8, "random")
    m = fv.Model(cfg, 64, FP32, theta)
    s = random_spins(64, cfg.n_spins, 3)
    a = to_np(m.log_prob(torch.as_tensor(s, device="cuda"))).astype(np.float64)
    b = to_np(m.log_prob_tokens(torch.as_tensor(((s + 1) // 2).astype(np.uint8), device="cuda"))).astype(np.float64)
    assert np.max(np.abs(a - b)) / cfg.n_spins <= 1e-6


def test_patched_model_refuses_the_single_spin_calls():
    cfg = ModelConfig(16, 32, 2, 2, vocab=16).with_mask(4, 4)
    theta = init_params(cfg, 1, "random")
    m = fv.Model(cfg, 8, FP32, theta)
    spins = torch.ones(8, 16, dtype=torch.int8, device="cuda")
    for call in (lambda: m.sample(8, 1, 1), lambda: m.log_prob(spins),
                 lambda: m.log_prob_backward(spins, torch.ones(8, device="cuda"))):
        with pytest.raises(fv.FvanError, match="patch tokens"):
            call()
    torch.cuda.synchronize()
    assert np.array_equal(to_np(m.params), theta.astype(np.float32))
    with pytest.raises(ValueError):
        m.log_prob_tokens(torch.zeros(8, 15, dtype=torch.uint8, device="cuda"))


def test_token_out_of_range_gives_nan_for_its_sample_only():
    cfg = ModelConfig(16, 32, 2, 2, vocab=16).with_mask(4, 4)
    theta = init_params(cfg, 2, "random")
    m = fv.Model(cfg, 6, FP32, theta)
    tok = _tokens(6, 16, 16, 9)
    clean = to_np(m.log_prob_tokens(torch.as_tensor(tok, device="cuda")))
    bad = tok.copy()
    bad[3, 7] = 200
    out = to_np(m.log_prob_tokens(torch.as_tensor(bad, device="cuda")))
    assert np.isnan(out[3])
    keep = np.arange(6) != 3
    assert np.array_equal(out[keep], clean[keep])
