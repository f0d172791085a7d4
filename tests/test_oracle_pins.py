"""Pins of the FP64 oracle to facts that do not come from the oracle itself:
printed numbers of the paper, published test vectors, closed forms, library
special cases, invariants and brute force on tiny inputs."""
import math
import os

import numpy as np
import pytest
import torch

from oracle import exact, markov, network as net, philox, physics, sampler, estimator
from workloads import ModelConfig, init_params, sk_instance, ea_instance
from workloads.instances import chain_instance, lattice_edges, random_spins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


# ---------------------------------------------------------------- generator

def test_philox_known_answers():
    for line in _rows("philox_kat.txt"):
        left, right = line.split("|")
        v = [int(x, 16) for x in left.split()]
        want = [int(x, 16) for x in right.split()]
        out = philox.philox4x32_10(np.array(v[:4], np.uint64), np.array(v[4:], np.uint64))
        assert [int(x) for x in out] == want


def test_uniform_draw_definition():
    u = philox.uniforms(seed=(7 << 32) | 11, stream=(3 << 32) | 5, batch=3, n=9, b0=2)
    for b in range(3):
        for t in range(9):
            w = philox.philox4x32_10(np.array([t >> 2, b + 2, 5, 3], np.uint64),
                                     np.array([11, 7], np.uint64))
            assert u[b, t] == (int(w[t & 3]) >> 8) / 2.0 ** 24
    assert u.min() >= 0.0 and u.max() < 1.0


# ---------------------------------------------------------------- architecture

def test_parameter_counts_match_paper():
    n = 0
    for line in _rows("param_counts.txt"):
        left = line.split("|")[0].split()
        S, V, dt, dp, nl, want = map(int, left)
        cfg = ModelConfig(n_spins=S, d_model=dt + dp, n_layers=nl, n_heads=1, d_token=dt, vocab=V)
        assert net.count(cfg) == want
        n += 1
    assert n == 14


def _theta(cfg, seed, style="random"):
    return net.as_theta(init_params(cfg, seed, style))


def test_visibility_definition_brute_force():
    for (n, W, P) in [(9, 2, 0), (9, 2, 3), (7, 6, 0), (8, 0, 0), (10, 3, 4)]:
        vis = net.visibility(n, W, P).numpy()
        for t in range(n):
            for j in range(n):
                assert vis[t, j] == (j <= t and (t - j <= W or j < P))


def test_blocks_match_library_transformer_layer():
    """Special case: a pre-LN torch TransformerEncoderLayer whose output projection is the
    identity (no W_O) and whose FFN is 4d wide with exact GELU computes one FlashVAN block."""
    cfg = ModelConfig(n_spins=11, d_model=32, n_layers=2, n_heads=2).with_mask(3, 2)
    th = _theta(cfg, 4)
    p = net.unflatten(th, cfg)
    spins = torch.as_tensor(random_spins(5, 11, 9))
    x = net.embed(p, cfg, net.tokens(spins), torch.arange(11))
    vis = net.visibility(11, cfg.window, cfg.prefix)
    d = cfg.d_model
    for l in range(cfg.n_layers):
        layer = torch.nn.TransformerEncoderLayer(d, cfg.n_heads, dim_feedforward=4 * d, dropout=0.0,
                                                 activation="gelu", norm_first=True, batch_first=True,
                                                 dtype=torch.float64)
        with torch.no_grad():
            layer.self_attn.in_proj_weight.copy_(p[f"l{l}.qkv.w"])
            layer.self_attn.in_proj_bias.copy_(p[f"l{l}.qkv.b"])
            layer.self_attn.out_proj.weight.copy_(torch.eye(d, dtype=torch.float64))
            layer.self_attn.out_proj.bias.zero_()
            layer.norm1.weight.copy_(p[f"l{l}.ln1.g"]); layer.norm1.bias.copy_(p[f"l{l}.ln1.b"])
            layer.norm2.weight.copy_(p[f"l{l}.ln2.g"]); layer.norm2.bias.copy_(p[f"l{l}.ln2.b"])
            layer.linear1.weight.copy_(p[f"l{l}.ffn1.w"]); layer.linear1.bias.copy_(p[f"l{l}.ffn1.b"])
            layer.linear2.weight.copy_(p[f"l{l}.ffn2.w"]); layer.linear2.bias.copy_(p[f"l{l}.ffn2.b"])
        layer.eval()
        with torch.no_grad():
            ref = layer(x, src_mask=~vis)
            mine = net.block(p, l, cfg, x, vis)
        assert torch.allclose(ref, mine, atol=1e-12, rtol=1e-12)
        x = mine
    z = x @ p["head.w"].T + p["head.b"]
    assert torch.allclose(z, net.logits(th, cfg, spins), atol=1e-12)


def test_full_causal_equals_library_attention():
    cfg = ModelConfig(n_spins=13, d_model=32, n_layers=1, n_heads=2).full_causal()
    g = torch.Generator().manual_seed(0)
    q, k, v = (torch.randn(3, 13, 32, generator=g, dtype=torch.float64) for _ in range(3))
    mine = net.masked_attention(q, k, v, net.visibility(13, 12, 0), 2)
    qh, kh, vh = (t.view(3, 13, 2, 16).transpose(1, 2) for t in (q, k, v))
    ref = torch.nn.functional.scaled_dot_product_attention(qh, kh, vh, is_causal=True)
    assert torch.allclose(mine, ref.transpose(1, 2).reshape(3, 13, 32), atol=1e-12)


def test_zero_layer_model_closed_form():
    """n_l = 0: p_t depends on the previous spin and the position only,
    z_t = W_h [T[tok_t]; P[t]] + b_h."""
    cfg = ModelConfig(n_spins=6, d_model=8, n_layers=0, n_heads=1).full_causal()
    th = init_params(cfg, 3, "random").astype(np.float64)
    T = th[:4].reshape(2, 2)
    P = th[4:4 + 36].reshape(6, 6)
    Wh = th[40:56].reshape(2, 8)
    bh = th[56:58]
    spins = random_spins(4, 6, 1)
    lp = net.log_p_sites(net.as_theta(th), cfg, spins).numpy()
    for b in range(4):
        for t in range(6):
            tok = 0 if t == 0 else (spins[b, t - 1] + 1) // 2
            z = Wh @ np.concatenate([T[tok], P[t]]) + bh
            s = (spins[b, t] + 1) // 2
            assert abs(lp[b, t] - (z[s] - np.log(np.exp(z).sum()))) < 1e-12


@pytest.mark.parametrize("W,P,n_l", [(9, 0, 2), (2, 0, 2), (2, 3, 2), (0, 0, 1), (3, 1, 3)])
def test_normalisation_by_enumeration(W, P, n_l):
    """sum_sigma q(sigma) = 1 for any parameters (autoregressive product, Eq. 11);
    a leaked future token or a wrong input shift breaks it."""
    cfg = ModelConfig(n_spins=10, d_model=32, n_layers=n_l, n_heads=2).with_mask(W, P)
    for seed, style in ((1, "random"), (2, "sharp")):
        _, lq = exact.enumerate_logq(init_params(cfg, seed, style), cfg)
        assert abs(np.exp(lq).sum() - 1.0) < 1e-12


def test_normalisation_sk16_model():
    cfg = ModelConfig(16, 32, 2, 2).full_causal()
    _, lq = exact.enumerate_logq(init_params(cfg, 7, "random"), cfg)
    assert abs(np.exp(lq).sum() - 1.0) < 1e-11


def test_conditionals_ignore_future_and_masked_past():
    cfg = ModelConfig(n_spins=12, d_model=32, n_layers=2, n_heads=2).with_mask(2, 2)
    th = _theta(cfg, 5)
    base = random_spins(1, 12, 3)
    ref = net.cond_plus(th, cfg, base).numpy()[0]
    vis = net.visibility(12, 2, 2).numpy()
    for t in range(12):
        for site in range(12):
            pos = site + 1                       # position carrying this site's token
            # a site feeds position t only through layers; with 2 layers the receptive
            # field is the 2-hop closure, so only check the definitely-invisible sites
            reach = np.linalg.matrix_power(vis.astype(int), 2)[t]
            if pos >= 12 or reach[pos] == 0:
                flip = base.copy()
                flip[0, site] *= -1
                assert abs(net.cond_plus(th, cfg, flip).numpy()[0, t] - ref[t]) < 1e-13


def test_one_layer_conditionals_depend_exactly_on_the_visible_sites():
    """One decoder layer: the conditional at position t reads the spin carried by
    key position j (site j - 1) only through attention, so it must change when
    that spin flips iff j <= t and (t - j <= W or j < P) -- the band of SI Eq. S1
    (A_tj = 0 only for t - j > W) plus the always-visible prefix (reading 11).
    Written from that statement, not from the oracle's mask: a band one key
    too narrow or too wide, or a lost prefix, fails here."""
    n, W, P = 14, 3, 2
    cfg = ModelConfig(n_spins=n, d_model=32, n_layers=1, n_heads=2).with_mask(W, P)
    th = _theta(cfg, 8)
    base = random_spins(1, n, 4)
    ref = net.cond_plus(th, cfg, base).numpy()[0]
    for site in range(n - 1):
        flip = base.copy()
        flip[0, site] *= -1
        got = net.cond_plus(th, cfg, flip).numpy()[0]
        j = site + 1
        for t in range(n):
            seen = j <= t and (t - j <= W or j < P)
            if seen:
                assert abs(got[t] - ref[t]) > 1e-9, (site, t)
            else:
                assert abs(got[t] - ref[t]) < 1e-13, (site, t)


# ---------------------------------------------------------------- energy

def _pair_loop_energy(sig, ei, ej, J):
    e = 0.0
    for a, b, c in zip(ei.tolist(), ej.tolist(), J.tolist()):
        e -= c * sig[a] * sig[b]
    return e


def test_energy_brute_force_and_symmetry():
    inst = ea_instance(4, 2, 11, "pm1")
    spins = random_spins(6, 16, 2)
    E = physics.energy_edges_int(spins, inst.edges_i, inst.edges_j, inst.J)
    for b in range(6):
        assert E[b] == _pair_loop_energy(spins[b].tolist(), inst.edges_i, inst.edges_j, inst.J)
    assert np.array_equal(E, physics.energy_edges_int(-spins, inst.edges_i, inst.edges_j, inst.J))
    assert np.all((E - inst.n_edges) % 2 == 0)          # sum of 2D*N/... +/-1 terms: parity of |E|
    sk = sk_instance(9, 3)
    s = random_spins(5, 9, 4)
    Ed = physics.energy_dense(s, sk.dense)
    Ee = physics.energy_edges(s, sk.edges_i, sk.edges_j, sk.J)
    assert np.allclose(Ed, Ee, atol=1e-12)
    for b in range(5):
        assert abs(Ee[b] - _pair_loop_energy(s[b].tolist(), sk.edges_i, sk.edges_j, sk.J)) < 1e-12


def test_lattice_edge_counts():
    assert lattice_edges(16, 2, True)[0].shape[0] == 512
    assert lattice_edges(10, 3, True)[0].shape[0] == 3000
    assert lattice_edges(32, 2, True)[0].shape[0] == 2048
    ei, ej = lattice_edges(5, 3, True)
    pairs = {tuple(sorted(p)) for p in zip(ei.tolist(), ej.tolist())}
    assert len(pairs) == ei.shape[0]                     # each unordered pair once


def test_sk_annealed_partition_function():
    """E_J[Z] = 2^N exp(beta^2 (N-1) / 4) when each pair i<j is counted once with
    Var(J_ij) = 1/N; counting pairs twice or dropping the 1/sqrt(N) changes the exponent."""
    n, beta, reps = 8, 0.7, 3000
    sig = physics.all_configs(n)
    Zs = []
    for r in range(reps):
        inst = sk_instance(n, 50_000 + r)
        Zs.append(np.exp(physics.log_partition(physics.energy_dense(sig, inst.dense), beta)))
    Zs = np.array(Zs)
    want = 2.0 ** n * math.exp(beta ** 2 * (n - 1) / 4)
    assert abs(Zs.mean() - want) < 4 * Zs.std() / math.sqrt(reps)
    wrong = 2.0 ** n * math.exp(beta ** 2 * (n - 1) / 2)
    assert abs(Zs.mean() - wrong) > 4 * Zs.std() / math.sqrt(reps)


def test_sk_free_energy_near_thermodynamic_limit():
    """Paper: F_inf ~ -1.5112 at beta = 0.5.  At N = 16 the quenched free energy per spin
    over instances must sit just above the annealed value -ln2/beta - beta (N-1)/(4N)
    (Jensen) and within finite-size distance of F_inf."""
    vals = dict(line.split() for line in _rows("sk_thermo.txt"))
    beta, f_inf = float(vals["beta"]), float(vals["f_inf"])
    assert abs(-math.log(2) / beta - beta / 4 - f_inf) < 1e-4
    n = 16
    sig = physics.all_configs(n)
    fs = [physics.free_energy_exact(physics.energy_dense(sig, sk_instance(n, 70_000 + r).dense), beta) / n
          for r in range(40)]
    annealed = -math.log(2) / beta - beta * (n - 1) / (4 * n)
    assert annealed - 1e-3 < np.mean(fs) < annealed + 0.01
    assert abs(np.mean(fs) - f_inf) < 0.02


# ---------------------------------------------------------------- estimator

def _chain_optimum(n, beta):
    """Parameters of a zero-layer model that equals the Boltzmann distribution of
    the open ferromagnetic chain E = -sum sigma_t sigma_{t+1}: p(sigma_0) = 1/2 and
    log-odds 2 beta sigma_{t-1} for t >= 1."""
    cfg = ModelConfig(n_spins=n, d_model=3, n_layers=0, n_heads=1, d_token=2).full_causal()
    th = np.zeros(net.count(cfg))
    T = np.array([[-1.0, 0.0], [1.0, 0.0]])              # token rows: sigma = -1, +1 (row 0 = start)
    Pe = np.zeros((n, 1))
    Pe[0, 0] = 1.0                                       # position 0 flag cancels the start token
    Wh = np.array([[-beta, 0.0, -beta], [beta, 0.0, beta]])
    th[:4] = T.ravel()
    th[4:4 + n] = Pe.ravel()
    th[4 + n:4 + n + 6] = Wh.ravel()
    return cfg, th


def test_chain_optimum_gives_exact_free_energy_and_zero_variance():
    n, beta = 10, 0.8
    cfg, th = _chain_optimum(n, beta)
    inst = chain_instance(n)
    sig = physics.all_configs(n)
    E = physics.energy_edges(sig, inst.edges_i, inst.edges_j, inst.J)
    Fq, F, qsum = exact.exact_free_energies(th, cfg, E, beta)
    F_closed = -(math.log(2) + (n - 1) * math.log(2 * math.cosh(beta))) / beta
    assert abs(F - F_closed) < 1e-12
    assert abs(Fq - F) < 1e-12 and abs(qsum - 1) < 1e-12
    spins, lq, _ = sampler.kv_sample(th, cfg, 200, 1, 2)
    Es = physics.energy_edges(spins, inst.edges_i, inst.edges_j, inst.J)
    mean, var = estimator.free_energy_stats(Es, lq, beta, n)
    assert abs(mean - F / n) < 1e-12 and var < 1e-24
    g = estimator.reinforce_gradient(th, cfg, spins, Es, lq, beta)
    assert np.abs(g).max() < 1e-12


def test_variational_bound_and_estimator_mean():
    """F_q >= F (Eq. 4) and the sample mean of f_b converges to F_q / N."""
    cfg = ModelConfig(n_spins=10, d_model=32, n_layers=2, n_heads=2).full_causal()
    th = init_params(cfg, 8, "random")
    inst = sk_instance(10, 17)
    beta = 1.3
    E_all = physics.energy_dense(physics.all_configs(10), inst.dense)
    Fq, F, _ = exact.exact_free_energies(th, cfg, E_all, beta)
    assert Fq >= F - 1e-12
    spins, lq, _ = sampler.kv_sample(th, cfg, 4000, 3, 4)
    E = physics.energy_dense(spins, inst.dense)
    mean, var = estimator.free_energy_stats(E, lq, beta, 10)
    assert abs(mean - Fq / 10) < 4 * math.sqrt(var / 4000)


def test_reinforce_estimator_is_unbiased_for_exact_gradient():
    """Batch-averaged REINFORCE gradient vs the enumerated grad F_q (Eq. 18), and the
    enumerated gradient vs reverse mode through F_q(theta) itself."""
    cfg = ModelConfig(n_spins=8, d_model=16, n_layers=1, n_heads=1).full_causal()
    th = init_params(cfg, 12, "random")
    inst = sk_instance(8, 5)
    beta = 1.0
    E_all = physics.energy_dense(physics.all_configs(8), inst.dense)
    g_exact = exact.exact_grad_Fq(th, cfg, E_all, beta)
    tt = net.as_theta(th, requires_grad=True)
    exact.Fq_function(tt, cfg, E_all, beta).backward()
    assert np.allclose(tt.grad.numpy(), g_exact, atol=1e-12, rtol=1e-9)
    B, reps = 512, 24
    gs = []
    for r in range(reps):
        spins, lq, _ = sampler.kv_sample(th, cfg, B, 100 + r, r)
        E = physics.energy_dense(spins, inst.dense)
        gs.append(estimator.reinforce_gradient(th, cfg, spins, E, lq, beta))
    gs = np.array(gs)
    mean, se = gs.mean(0), gs.std(0, ddof=1) / math.sqrt(reps) + 1e-12
    idx = np.argsort(-np.abs(g_exact))[:40]
    z = (mean[idx] - g_exact[idx]) / se[idx]
    assert np.mean(np.abs(z) < 3.5) > 0.9
    cos = mean @ g_exact / (np.linalg.norm(mean) * np.linalg.norm(g_exact))
    assert cos > 0.9


def test_surrogate_gradient_matches_finite_differences():
    cfg = ModelConfig(n_spins=12, d_model=32, n_layers=2, n_heads=2).with_mask(3, 2)
    th = init_params(cfg, 21, "random").astype(np.float64)
    spins = random_spins(6, 12, 8)
    c = np.random.default_rng(1).standard_normal(6)
    g = estimator.grad_surrogate(th, cfg, spins, c)
    rng = np.random.default_rng(2)
    idx = rng.choice(th.shape[0], 64, replace=False)
    h = 1e-5
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        sp = float(estimator.surrogate(net.as_theta(tp), cfg, spins, c))
        sm = float(estimator.surrogate(net.as_theta(tm), cfg, spins, c))
        fd = (sp - sm) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 + 1e-6 * abs(g[k])


def test_adam_matches_library_optimizer():
    rng = np.random.default_rng(0)
    th = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.tensor(th))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    cur = th.copy()
    for step in range(1, 6):
        g = rng.standard_normal(50)
        p.grad = torch.tensor(g)
        opt.step()
        cur, m, v = estimator.adam_update(cur, g, m, v, step, 1e-2)
    assert np.allclose(cur, p.detach().numpy(), atol=1e-13)


# ---------------------------------------------------------------- sampling

def test_kv_cache_sampler_matches_naive_and_teacher_forcing():
    cfg = ModelConfig(n_spins=14, d_model=32, n_layers=2, n_heads=2).with_mask(3, 4)
    th = init_params(cfg, 31, "random")
    s1, l1, pp = sampler.kv_sample(th, cfg, 48, 9, 1)
    s2, l2 = sampler.naive_sample(th, cfg, 48, 9, 1)
    assert np.array_equal(s1, s2)
    assert np.abs(l1 - l2).max() < 1e-12
    tf = net.log_q(net.as_theta(th), cfg, s1).numpy()
    assert np.abs(l1 - tf).max() < 1e-12
    bad, _, _ = sampler.decision_check(th, cfg, s1, 9, 1, tol=0.0)
    assert bad == 0


def test_sample_frequencies_follow_q():
    cfg = ModelConfig(n_spins=6, d_model=16, n_layers=1, n_heads=1).full_causal()
    th = init_params(cfg, 2, "random")
    sig, lq = exact.enumerate_logq(th, cfg)
    B = 20000
    spins, _, _ = sampler.kv_sample(th, cfg, B, 77, 0)
    idx = ((spins > 0).astype(np.int64) * (1 << np.arange(5, -1, -1))).sum(1)
    counts = np.bincount(idx, minlength=64)
    expect = B * np.exp(lq)
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 63 + 5 * math.sqrt(2 * 63)


# ---------------------------------------------------------------- Markov boundary

@pytest.mark.parametrize("L,pbc", [(4, False), (4, True), (3, True)])
def test_markov_boundary_brute_force(L, pbc):
    ei, ej = lattice_edges(L, 2, pbc)
    J = np.random.default_rng(L + 10 * pbc).standard_normal(ei.shape[0])
    n = L * L
    assert markov.brute_force_dependence(n, ei, ej, J, 0.9) == markov.ordered_boundary(n, ei, ej)


def test_mask_rule_on_workload_lattices():
    want = {(16, 2, True): (16, 17), (10, 3, True): (100, 101), (32, 2, True): (32, 33),
            (24, 2, True): (24, 25), (6, 2, False): (6, 0), (4, 3, False): (16, 0)}
    for (L, D, pbc), (W, P) in want.items():
        ei, ej = lattice_edges(L, D, pbc)
        assert markov.derive_mask(L ** D, ei, ej) == (W, P)
        bnd = markov.ordered_boundary(L ** D, ei, ej)
        assert markov.mask_covers(L ** D, bnd, W, P)
    sk = sk_instance(12, 0)
    assert markov.derive_mask(12, sk.edges_i, sk.edges_j) == (11, 0)


def test_sparse_mask_is_exact_for_boltzmann_conditionals():
    """With the derived (W, P), zeroing what the mask hides cannot change an exact
    conditional: each conditional depends only on sites the mask keeps visible."""
    for pbc in (False, True):
        ei, ej = lattice_edges(4, 2, pbc)
        J = np.random.default_rng(5).standard_normal(ei.shape[0])
        W, P = markov.derive_mask(16, ei, ej)
        deps = markov.brute_force_dependence(16, ei, ej, J, 1.1)
        for i in range(16):
            for j in deps[i]:
                pos = j + 1
                assert i - pos <= W or pos < P
