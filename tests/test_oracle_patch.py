"""Pins of the oracle's 2^D patching (oracle.patch) to facts outside it: the
patch geometry by brute force over lattice coordinates, the spin <-> token
bijection over every state, normalisation of the patched q by exhaustive
enumeration, the draw rule against its interval definition, reduction of the
V = 2 case to the binary sampler (pinned elsewhere), and the sampled
frequencies against q."""
import numpy as np
import pytest

from oracle import patch, sampler
from workloads import ModelConfig, init_params
from workloads.instances import random_spins


@pytest.mark.parametrize("L,D", [(2, 1), (6, 1), (4, 2), (6, 2), (4, 3)])
def test_patch_geometry_by_coordinates(L, D):
    """Every site sits in exactly one patch; bit m of patch t is the site whose
    coordinates are 2 P + o, P the patch's coordinates and o the offset of m."""
    sites = patch.patch_sites(L, D)
    P = L // 2
    assert sites.shape == (P ** D, 2 ** D)
    assert np.array_equal(np.sort(sites.reshape(-1)), np.arange(L ** D))
    for t in range(P ** D):
        pc = [(t // P ** (D - 1 - k)) % P for k in range(D)]
        for m in range(2 ** D):
            oc = [(m >> (D - 1 - k)) & 1 for k in range(D)]
            coords = [2 * pc[k] + oc[k] for k in range(D)]
            site = sum(c * L ** (D - 1 - k) for k, c in enumerate(coords))
            assert sites[t, m] == site


def test_worked_example_4x4():
    """One up spin at row r, column c of a 4x4 lattice (all others down) is token
    2^((r%2)*2 + c%2) at patch (r//2)*2 + c//2, and token 0 elsewhere."""
    for r in range(4):
        for c in range(4):
            s = -np.ones((1, 16), dtype=np.int8)
            s[0, 4 * r + c] = 1
            tok = patch.spins_to_tokens(s, 4, 2)[0]
            want = np.zeros(4, dtype=np.int64)
            want[(r // 2) * 2 + c // 2] = 1 << ((r % 2) * 2 + c % 2)
            assert np.array_equal(tok, want)
    assert np.array_equal(patch.spins_to_tokens(np.ones((1, 16), np.int8), 4, 2)[0], [15] * 4)


@pytest.mark.parametrize("L,D", [(4, 2), (2, 3)])
def test_tokens_are_a_bijection_of_spin_states(L, D):
    n = L ** D
    idx = np.arange(2 ** n, dtype=np.int64)
    spins = (2 * ((idx[:, None] >> np.arange(n)) & 1) - 1).astype(np.int8)
    tok = patch.spins_to_tokens(spins, L, D)
    V = 2 ** (2 ** D)
    assert tok.min() >= 0 and tok.max() < V
    code = np.zeros(len(idx), dtype=np.int64)
    for t in range(tok.shape[1]):
        code = code * V + tok[:, t]
    assert len(np.unique(code)) == 2 ** n
    assert np.array_equal(patch.tokens_to_spins(tok, L, D), spins)


def test_patched_q_is_normalised_over_all_spin_states():
    """4x4 lattice, 2x2 patches: 4 positions, vocabulary 16; sum over all 2^16
    spin configurations of q = 1, with and without a band mask."""
    n = 16
    idx = np.arange(2 ** n, dtype=np.int64)
    spins = (2 * ((idx[:, None] >> np.arange(n)) & 1) - 1).astype(np.int8)
    for cfg in (ModelConfig(4, 16, 2, 2, vocab=16).full_causal(), ModelConfig(4, 16, 2, 2, vocab=16).with_mask(1, 1)):
        theta = init_params(cfg, 5, "random")
        lq = patch.log_q_spins(theta, cfg, spins, 4, 2, chunk=1 << 14)
        assert abs(np.exp(lq).sum() - 1.0) < 1e-10


def test_draw_matches_its_interval_definition():
    rng = np.random.default_rng(2)
    for V in (2, 4, 16, 256):
        p = rng.dirichlet(np.full(V, 0.3), size=400)
        u = rng.random(400)
        tok = patch.categorical_draw(p, u)
        for b in range(400):
            above = p[b, tok[b] + 1:].sum()
            assert above <= u[b] < above + p[b, tok[b]] + 1e-15
    # a uniform grid of u reproduces p exactly in the limit of fine grids
    p = np.array([[0.125, 0.25, 0.5, 0.125]])
    u = (np.arange(1024) + 0.5) / 1024
    tok = patch.categorical_draw(np.repeat(p, 1024, axis=0), u)
    assert np.array_equal(np.bincount(tok, minlength=4) / 1024, p[0])


def test_vocabulary_two_is_the_binary_sampler():
    """Without patching (V = 2) the patched sampler is the pinned binary one: same
    uniforms, same spins, same ln q."""
    cfg = ModelConfig(9, 16, 2, 2).with_mask(3, 2)
    theta = init_params(cfg, 8, "random")
    tok, lq = patch.sample(theta, cfg, 32, seed=17, stream=4)
    spins, lq2 = sampler.naive_sample(theta, cfg, 32, seed=17, stream=4)[:2]
    assert np.array_equal(2 * tok - 1, spins)
    assert np.allclose(lq, lq2, rtol=0, atol=1e-12)


def test_sampler_log_q_is_the_teacher_forced_one():
    cfg = ModelConfig(9, 16, 2, 2, vocab=16).with_mask(2, 1)      # 6x6 lattice, 2x2 patches
    theta = init_params(cfg, 6, "random")
    tok, lq = patch.sample(theta, cfg, 24, seed=3, stream=1)
    assert np.allclose(lq, patch.log_q_tokens(theta, cfg, tok), rtol=0, atol=1e-12)
    spins = patch.tokens_to_spins(tok, 6, 2)
    assert np.array_equal(patch.spins_to_tokens(spins, 6, 2), tok)
    assert np.allclose(patch.log_q_spins(theta, cfg, spins, 6, 2), lq, rtol=0, atol=1e-12)


def test_sampled_frequencies_follow_q():
    """Two positions of vocabulary 16 (256 sequences): the counts of 40000 draws
    against 40000 q(seq), chi-square over all 256 sequences."""
    cfg = ModelConfig(2, 16, 1, 2, vocab=16).full_causal()
    theta = init_params(cfg, 12, "random")
    B = 40000
    tok, _ = patch.sample(theta, cfg, B, seed=99, stream=2)
    allseq = np.stack(np.meshgrid(np.arange(16), np.arange(16), indexing="ij"), -1).reshape(-1, 2)
    q = np.exp(patch.log_q_tokens(theta, cfg, allseq, chunk=256))
    assert abs(q.sum() - 1) < 1e-12
    cnt = np.bincount(tok[:, 0] * 16 + tok[:, 1], minlength=256)
    keep = B * q > 5
    chi2 = float(((cnt[keep] - B * q[keep]) ** 2 / (B * q[keep])).sum())
    k = int(keep.sum())
    assert chi2 < k + 6 * np.sqrt(2 * k)
    # drawing from the bottom of the vocabulary instead gives other tokens
    rev = patch.categorical_draw(np.full((1, 16), 1 / 16), np.array([0.01]))
    assert rev[0] == 15


def test_random_spins_round_trip_3d():
    s = random_spins(7, 6 ** 3, 4)
    tok = patch.spins_to_tokens(s, 6, 3)
    assert tok.shape == (7, 27) and tok.max() < 256
    assert np.array_equal(patch.tokens_to_spins(tok, 6, 3), s)


@pytest.mark.parametrize("L,D", [(4, 2), (8, 2), (6, 3), (10, 3)])
def test_patch_graph_of_the_inputs_by_brute_force(L, D):
    """The patch graph the benchmark derives its mask from (workloads.patch_edges)
    joins exactly the patches whose sites are lattice neighbours, found here by a
    brute-force pass over the oracle's patch geometry."""
    from workloads.instances import lattice_edges, patch_edges
    T, pi, pj = patch_edges(L, D)
    sites = patch.patch_sites(L, D)
    assert T == sites.shape[0]
    owner = {int(s): t for t in range(T) for s in sites[t]}
    ei, ej = lattice_edges(L, D, True)
    want = {tuple(sorted((owner[int(a)], owner[int(b)]))) for a, b in zip(ei, ej) if owner[int(a)] != owner[int(b)]}
    got = list(zip(pi.tolist(), pj.tolist()))
    assert len(got) == len(set(got)) and set(got) == want
    assert all(a < b for a, b in got)


def test_token_gradient_by_central_differences():
    """The patched model's reverse-mode gradient of sum_b c_b ln q(tok_b) against
    central differences of the same FP64 sum on coordinates spread over every
    parameter block (token table, positions, every layer, head)."""
    cfg = ModelConfig(6, 32, 2, 2, vocab=16).with_mask(2, 1)
    theta = init_params(cfg, 4, "random")
    rng = np.random.default_rng(2)
    tok = rng.integers(0, 16, size=(5, 6))
    c = rng.standard_normal(5)
    g = patch.grad_surrogate_tokens(theta, cfg, tok, c)

    def f(th):
        return float(np.dot(c, patch.log_q_tokens(th, cfg, tok)))

    idx = np.unique(np.concatenate([rng.integers(0, theta.size, 40), [0, 5, 31, theta.size - 1, theta.size - 20]]))
    h = 1e-6
    for i in idx:
        tp, tm = theta.astype(np.float64).copy(), theta.astype(np.float64).copy()
        tp[i] += h
        tm[i] -= h
        fd = (f(tp) - f(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
