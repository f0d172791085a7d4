"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol include/fvan.h declares, and its host logic (parameter count, mask
derivation, argument checks) agrees with the oracle and the paper."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2606_22984_amd as fv
from oracle import markov, network as net
from workloads import ModelConfig, sk_instance
from workloads.instances import lattice_edges

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "fvan.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"\b(?:int|const char\*)\s+(fvan_\w+)\s*\(", hdr))
    assert declared == set(fv.EXPORTS)
    lib = fv.lib()
    for name in declared:
        assert hasattr(lib, name), name


def test_num_params_matches_paper_counts():
    here = os.path.join(ROOT, "tests", "golden", "param_counts.txt")
    rows = [l.split("|")[0].split() for l in open(here) if l.strip() and not l.startswith("#")]
    for S, V, dt, dp, nl, want in (map(int, r) for r in rows):
        c = fv.ModelConfigC(n_spins=S, d_model=dt + dp, d_token=dt, n_layers=nl, n_heads=1, vocab=V,
                            window=0, prefix=0, max_batch=1, precision=0)
        out = C.c_int64()
        assert fv.lib().fvan_num_params(C.byref(c), C.byref(out)) == 0
        assert out.value == want


def test_num_params_matches_oracle_layout():
    for cfg in (ModelConfig(16, 32, 2, 2), ModelConfig(1000, 128, 8, 8), ModelConfig(256, 64, 4, 4)):
        assert fv.num_params(cfg) == net.count(cfg)


@pytest.mark.parametrize("L,D,pbc", [(16, 2, True), (10, 3, True), (24, 2, True), (32, 2, True),
                                     (6, 2, False), (4, 3, False), (5, 2, True)])
def test_mask_derivation_matches_oracle(L, D, pbc):
    ei, ej = lattice_edges(L, D, pbc)
    assert fv.derive_mask(L ** D, ei, ej) == markov.derive_mask(L ** D, ei, ej)


def test_mask_derivation_sk_and_errors():
    sk = sk_instance(20, 1)
    assert fv.derive_mask(20, sk.edges_i, sk.edges_j) == (19, 0)
    with pytest.raises(fv.FvanError) as e:
        fv.derive_mask(4, [0, 1], [1, 7])
    assert e.value.code == -1


def test_invalid_configs_are_rejected_on_the_host():
    base = dict(n_spins=16, d_model=32, d_token=2, n_layers=2, n_heads=2, vocab=2, window=15, prefix=0,
                max_batch=8, precision=0)
    bad = [dict(d_model=48), dict(n_heads=4), dict(n_heads=3), dict(vocab=1), dict(vocab=257), dict(window=-1),
           dict(prefix=17), dict(max_batch=0), dict(precision=7), dict(precision=1), dict(workspaces=4)]
    for b in bad:
        c = fv.ModelConfigC(**{**base, **b})
        h = C.c_void_p()
        rc = fv.lib().fvan_create_model(C.byref(c), C.byref(h))
        assert rc in (-1, -5), b
        assert not h.value
        assert fv.lib().fvan_last_error()


def test_null_arguments_are_rejected():
    lib = fv.lib()
    assert lib.fvan_sample(None, 1, 0, 0, None, None, None) == -1
    assert lib.fvan_energy(None, 1, None, None, None) == -1
    assert lib.fvan_free_energy(4, 4, 1.0, 0, None, None, None, None) == -1
    assert lib.fvan_free_energy(4, 4, -1.0, 0, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None) == -1
    assert lib.fvan_reinforce_weights(0, 1.0, 0, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None) == -1
    assert lib.fvan_destroy_model(None) == -1


def test_newton_schulz_and_muon_argument_checks():
    """Rejected on the host before anything is enqueued (no GPU needed)."""
    lib, p = fv.lib(), C.c_void_p(8)
    f = C.c_float
    assert lib.fvan_newton_schulz(0, 4, 5, f(1e-7), p, p, None) == -1
    assert lib.fvan_newton_schulz(4, -1, 5, f(1e-7), p, p, None) == -1
    assert lib.fvan_newton_schulz(129, 200, 5, f(1e-7), p, p, None) == -1
    assert lib.fvan_newton_schulz(200, 129, 5, f(1e-7), p, p, None) == -1
    assert lib.fvan_newton_schulz(1 << 7, 1 << 24, 5, f(1e-7), p, p, None) == -1
    assert lib.fvan_newton_schulz(8, 8, 17, f(1e-7), p, p, None) == -1
    assert lib.fvan_newton_schulz(8, 8, -1, f(1e-7), p, p, None) == -1
    assert lib.fvan_newton_schulz(8, 8, 5, f(0.0), p, p, None) == -1
    assert lib.fvan_newton_schulz(8, 8, 5, f(float("inf")), p, p, None) == -1
    assert lib.fvan_newton_schulz(8, 8, 5, f(1e-7), None, p, None) == -1
    assert "Newton-Schulz" in lib.fvan_last_error().decode() or "eps" in lib.fvan_last_error().decode() \
        or "NULL" in lib.fvan_last_error().decode()
    o = fv.muon_struct()
    assert lib.fvan_muon_step(None, C.byref(o), 1, None) == -1
    assert lib.fvan_train_step_muon(None, None, 1.0, 1, 0, 1, C.byref(o), None, None) == -1


def test_refinement_argument_checks():
    lib, p = fv.lib(), C.c_void_p(8)
    g = fv.LmcC(degree=4, nbr=8, J=8, colour=8, sweeps=1)
    assert lib.fvan_lmc_refine(16, C.byref(g), 4, 1.0, 0, 0, None, None, None) == -1      # NULL spins
    assert lib.fvan_lmc_refine(0, C.byref(g), 4, 1.0, 0, 0, p, None, None) == -1
    assert lib.fvan_lmc_refine(16385, C.byref(g), 4, 1.0, 0, 0, p, None, None) == -1
    assert lib.fvan_lmc_refine(16, C.byref(g), 4, float("nan"), 0, 0, p, None, None) == -1
    assert lib.fvan_lmc_refine(16, C.byref(g), 4, -1.0, 0, 0, p, None, None) == -1
    bad = fv.LmcC(degree=0, nbr=8, J=8, colour=8, sweeps=1)
    assert lib.fvan_lmc_refine(16, C.byref(bad), 4, 1.0, 0, 0, p, None, None) == -1
    nul = fv.LmcC(degree=4, nbr=None, J=8, colour=8, sweeps=1)
    assert lib.fvan_lmc_refine(16, C.byref(nul), 4, 1.0, 0, 0, p, None, None) == -1
    assert lib.fvan_distill_weights(4, 1.0, 0.1, 0, None, p, p, None) == -1
    assert lib.fvan_distill_weights(4, 0.0, 0.1, 0, p, p, p, None) == -1
    assert lib.fvan_train_step_distill(None, None, None, 1.0, 0.1, 1, 0, 1, None, None, None) == -1


def test_annealing_schedule_matches_oracle():
    """Host-only entry point: the library's schedule equals the oracle's at every step."""
    from oracle import overlap
    for T0, nw, neq, na in [(2.0, 1200, 5, 500), (1.5, 0, 1, 7), (0.3, 10, 3, 4)]:
        for i in list(range(0, nw + neq * na + 12)) if nw < 100 else list(range(0, 4000, 7)):
            assert fv.anneal_temperature(i, T0, nw, neq, na) == overlap.anneal_temperature(i, T0, nw, neq, na)
    lib = fv.lib()
    T = C.c_double()
    assert lib.fvan_anneal_temperature(1, 0.0, 0, 1, 1, C.byref(T)) == -1
    assert lib.fvan_anneal_temperature(1, 1.0, 0, 0, 1, C.byref(T)) == -1
    assert lib.fvan_anneal_temperature(1, 1.0, 0, 1, 0, C.byref(T)) == -1
    assert lib.fvan_anneal_temperature(1, 1.0, -1, 1, 1, C.byref(T)) == -1


def test_overlap_histogram_argument_checks():
    lib, p = fv.lib(), C.c_void_p(8)
    assert lib.fvan_overlap_histogram(4, 10, None, p, None) == -1
    assert lib.fvan_overlap_histogram(0, 10, p, p, None) == -1
    assert lib.fvan_overlap_histogram((1 << 20) + 1, 10, p, p, None) == -1
    assert lib.fvan_overlap_histogram(4, 16001, p, p, None) == -1


def test_model_status_and_group_argument_checks():
    lib = fv.lib()
    assert lib.fvan_model_status(None, None) == -1
    assert lib.fvan_group_create(None, 1, 0, None) == -1


def test_refinement_graph_needs_a_proper_colouring():
    """Odd L under periodic boundaries puts the neighbours x = L-1 and x = 0 in one
    checkerboard colour: the graph builder refuses it (host only, CPU tensors)."""
    from workloads import ea_instance
    g = fv.lmc_graph(ea_instance(6, 2, 1, "pm1"), 1, device="cpu")
    assert g.colour.shape == (36,)
    for L, dim in ((5, 2), (3, 3)):
        with pytest.raises(ValueError, match="colouring"):
            fv.lmc_graph(ea_instance(L, dim, 1, "pm1"), 1, device="cpu")
    fv.lmc_graph(ea_instance(5, 2, 1, "pm1", pbc=False), 1, device="cpu")   # open boundaries: bipartite


def test_token_entry_points_reject_bad_arguments_on_the_host():
    lib, p = fv.lib(), C.c_void_p(8)
    assert lib.fvan_sample_tokens(None, 1, 0, 0, p, p, None) == -1
    assert lib.fvan_log_prob_tokens_backward(None, 1, p, p, None) == -1
    # tokens -> spins: n_tokens * bits must be n_spins, bits in [1, 8]
    assert lib.fvan_tokens_to_spins(16, 4, p, 63, 1, p, p, None) == -1
    assert lib.fvan_tokens_to_spins(16, 9, p, 144, 1, p, p, None) == -1
    assert lib.fvan_tokens_to_spins(16, 4, None, 64, 1, p, p, None) == -1
    assert lib.fvan_tokens_to_spins(16, 4, p, 64, 0, p, p, None) == -1
    o = fv.muon_struct()
    assert lib.fvan_train_step_tokens(None, None, p, 1.0, 1, 0, 1, C.byref(o), p, None) == -1
    assert lib.fvan_sample_noalloc(None, 1, 0, 0, p, p, None) == -1
    assert lib.fvan_group_launch_shape(None, None, None, None, None) == -1


def test_binding_patch_geometry_equals_the_oracles():
    """The binding's site map of patch tokens (its own code) against the oracle's."""
    from oracle import patch
    for L, D in ((2, 1), (6, 1), (4, 2), (8, 2), (4, 3), (10, 3)):
        assert np.array_equal(fv.patch_sites(L, D), patch.patch_sites(L, D)), (L, D)
    with pytest.raises(ValueError):
        fv.patch_sites(5, 2)
