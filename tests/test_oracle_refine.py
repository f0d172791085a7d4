"""Pins of the oracle's local Monte Carlo refinement and self-distillation
weights (oracle.refine) to facts outside it: flip energies by brute force, the
beta = 0 closed form, stationarity of the Boltzmann distribution (exact
enumeration on a 4x4 lattice), the zero-temperature descent property, and the
sum rule of the weights."""
import numpy as np

from oracle import estimator, physics, refine
from workloads import ea_instance
from workloads.instances import random_spins


def _inst(L=4, dim=2, seed=3, bonds="gauss"):
    inst = ea_instance(L, dim, seed, bonds)
    return inst, refine.neighbours(inst.n, inst.edges_i, inst.edges_j, inst.J), refine.checkerboard_colour(L, dim)


def test_colouring_is_proper_on_even_periodic_lattices():
    for L, dim in [(4, 2), (6, 2), (4, 3), (10, 3)]:
        inst = ea_instance(L, dim, 1, "pm1")
        c = refine.checkerboard_colour(L, dim)
        assert np.all(c[inst.edges_i] != c[inst.edges_j])
        assert c.sum() == inst.n // 2


def test_flip_energy_is_twice_spin_times_local_field():
    inst, adj, _ = _inst()
    s = random_spins(5, inst.n, 11)
    h = refine.local_fields(s, adj)
    E0 = physics.energy_edges(s, inst.edges_i, inst.edges_j, inst.J)
    for i in range(inst.n):
        t = s.copy()
        t[:, i] = -t[:, i]
        dE = physics.energy_edges(t, inst.edges_i, inst.edges_j, inst.J) - E0
        assert np.allclose(dE, 2.0 * s[:, i] * h[:, i], rtol=0, atol=1e-12)


def test_beta_zero_flips_every_spin_once_per_sweep():
    inst, adj, col = _inst()
    s = random_spins(4, inst.n, 2)
    out, acc = refine.metropolis_checkerboard(s, adj, col, 0.0, 1, seed=5, stream=1)
    assert np.array_equal(out, -s) and np.all(acc == inst.n)
    out2, _ = refine.metropolis_checkerboard(s, adj, col, 0.0, 2, seed=5, stream=1)
    assert np.array_equal(out2, s)


def test_zero_temperature_sweeps_never_raise_the_energy():
    inst, adj, col = _inst(6, 2, 4)
    s = random_spins(64, inst.n, 3)
    E = physics.energy_edges(s, inst.edges_i, inst.edges_j, inst.J)
    for k in range(4):
        s, _ = refine.metropolis_checkerboard(s, adj, col, 1e6, 1, seed=9, stream=k)
        E1 = physics.energy_edges(s, inst.edges_i, inst.edges_j, inst.J)
        assert np.all(E1 <= E + 1e-9)
        E = E1


def test_checkerboard_sweeps_keep_the_boltzmann_distribution():
    """Exact samples of exp(-beta E)/Z on a 4x4 periodic lattice stay Boltzmann
    distributed after sweeps: the energy histogram matches the enumerated one."""
    inst, adj, col = _inst(4, 2, 8)
    beta = 0.9
    allc = physics.all_configs(inst.n)
    E_all = physics.energy_edges(allc, inst.edges_i, inst.edges_j, inst.J)
    p = np.exp(-beta * (E_all - E_all.min()))
    p /= p.sum()
    rng = np.random.default_rng(0)
    B = 60000
    s0 = allc[rng.choice(allc.shape[0], size=B, p=p)]
    s, _ = refine.metropolis_checkerboard(s0, adj, col, beta, 3, seed=123, stream=7)
    E = physics.energy_edges(s, inst.edges_i, inst.edges_j, inst.J)
    mean_exact = float((p * E_all).sum())
    sd = float(np.sqrt((p * (E_all - mean_exact) ** 2).sum()))
    assert abs(E.mean() - mean_exact) < 4 * sd / np.sqrt(B)
    # the same at the level of individual states (chi-square over the 64 likeliest)
    top = np.argsort(-p)[:64]
    code = (((s > 0).astype(np.int64)) << np.arange(inst.n - 1, -1, -1)[None, :]).sum(axis=1)
    cnt = np.bincount(code, minlength=allc.shape[0])[top]
    expct = B * p[top]
    chi2 = float(((cnt - expct) ** 2 / expct).sum())
    assert chi2 < 64 + 6 * np.sqrt(2 * 64)
    # a wrong acceptance sign heats the samples far beyond that
    bad, _ = refine.metropolis_checkerboard(s0, adj, col, -beta, 3, seed=123, stream=7)
    Eb = physics.energy_edges(bad, inst.edges_i, inst.edges_j, inst.J)
    assert Eb.mean() - mean_exact > 20 * sd / np.sqrt(B)


def test_distill_weights_sum_rule_and_reinforce_limit():
    rng = np.random.default_rng(4)
    E, lq = rng.standard_normal(33) * 5, rng.standard_normal(33) * 3 - 10
    for w in (0.0, 0.3, 2.0):
        c = refine.distill_weights(E, lq, 0.7, w)
        assert abs(c.sum() + w / 0.7) < 1e-12           # the likelihood term carries the 1/beta too
    assert np.allclose(refine.distill_weights(E, lq, 0.7, 0.0), estimator.reinforce_weights(E, lq, 0.7),
                       rtol=0, atol=1e-15)
