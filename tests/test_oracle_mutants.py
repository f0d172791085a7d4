"""Planted mistakes in the oracle.  Each mutant is the oracle with one plausible
error written into its source (a dropped term, a wrong sign or index, a
transposed order, a wrong constant); each must fail at least one of the pins
that tie the oracle to the paper and to the mathematics (the pin tests of the
other oracle test modules, run here against the mutant).  A mutant that passes
every pin listed for it would show a blind spot of the pins."""
import inspect
import textwrap

import pytest

from oracle import muon, network, overlap, patch, refine
from tests import test_oracle_muon as pin_muon
from tests import test_oracle_overlap as pin_overlap
from tests import test_oracle_patch as pin_patch
from tests import test_oracle_pins as pin_core
from tests import test_oracle_refine as pin_refine


def mutant(module, fname, old, new):
    """module.fname with its source text `old` replaced by `new` (which must occur)."""
    src = textwrap.dedent(inspect.getsource(getattr(module, fname)))
    assert old in src, (fname, old)
    ns = dict(vars(module))
    exec(compile(src.replace(old, new), f"<mutant of {module.__name__}.{fname}>", "exec"), ns)
    return ns[fname]


def killed(pins) -> bool:
    for pin in pins:
        try:
            pin()
        except AssertionError:
            return True
    return False


# (description, module, function, old text, new text, pins)
MUTANTS = [
    # overlap histogram and annealing schedule
    ("agreement counted from the wrong end", overlap, "overlap_counts", "k = (Q[a, b] + N) // 2",
     "k = (N - Q[a, b]) // 2", [pin_overlap.test_all_configurations_closed_form]),
    ("diagonal pairs included", overlap, "overlap_counts", "np.triu_indices(B, k=1)", "np.triu_indices(B, k=0)",
     [pin_overlap.test_all_configurations_closed_form, pin_overlap.test_brute_force_pair_loop_and_flip_relation]),
    ("schedule floor off by one", overlap, "anneal_temperature", "(i - n_warmup) // n_eq, n_anneal",
     "(i - n_warmup) // n_eq + 1, n_anneal", [pin_overlap.test_annealing_schedule_endpoints]),
    # local Monte Carlo refinement and the Eq. (loss2) weights
    ("sign of the flip energy", refine, "metropolis_checkerboard", "dE = 2.0 * s * h", "dE = -2.0 * s * h",
     [pin_refine.test_zero_temperature_sweeps_never_raise_the_energy]),
    ("colour ignored (every site in every half-sweep)", refine, "metropolis_checkerboard",
     "mine = colour[None, :] == c", "mine = colour[None, :] >= 0",
     [pin_refine.test_beta_zero_flips_every_spin_once_per_sweep]),
    ("field taken from the site itself", refine, "local_fields", "h[:, i] += v * s[:, j]",
     "h[:, i] += v * s[:, i]", [pin_refine.test_flip_energy_is_twice_spin_times_local_field]),
    ("sign of the likelihood term", refine, "distill_weights", "((L - L.mean()) - w)", "((L - L.mean()) + w)",
     [pin_refine.test_distill_weights_sum_rule_and_reinforce_limit]),
    # Muon
    ("A instead of A^2 in the quintic", muon, "newton_schulz", "c * (A @ A)", "c * A",
     [pin_muon.test_newton_schulz_rank_one_closed_form]),
    ("sign of the polynomial term", muon, "newton_schulz", "X = a * X + B @ X", "X = a * X - B @ X",
     [pin_muon.test_newton_schulz_rank_one_closed_form]),
    ("max-norm for the Frobenius norm", muon, "newton_schulz", "np.linalg.norm(X)", "np.abs(X).max()",
     [lambda: pin_muon.test_newton_schulz_acts_on_singular_values(16, 48, 1)]),
    ("momentum order", muon, "muon_update", "M = momentum * m[sl] + grad[sl]", "M = m[sl] + momentum * grad[sl]",
     [pin_muon.test_muon_two_steps_closed_form]),
    ("sqrt of min(rows, cols) for max", muon, "muon_update", "math.sqrt(max(shape))", "math.sqrt(min(shape))",
     [pin_muon.test_muon_takes_exactly_the_layer_matrices]),
    # 2^D patching
    ("bit order inside a token reversed", patch, "patch_sites",
     "enumerate(itertools.product(range(2), repeat=D))",
     "enumerate(reversed(list(itertools.product(range(2), repeat=D))))", [pin_patch.test_worked_example_4x4]),
    ("draw walks the vocabulary from the bottom", patch, "categorical_draw", "for k in range(V - 1, 0, -1):",
     "for k in range(0, V - 1):", [pin_patch.test_draw_matches_its_interval_definition]),
    ("input tokens not shifted", patch, "input_tokens", "torch.cat([start, tok[:, :-1]], dim=1)", "tok",
     [pin_patch.test_patched_q_is_normalised_over_all_spin_states]),
    # the network itself
    ("spin tokens not shifted (site t sees its own spin)", network, "tokens",
     "torch.cat([start, s[:, :-1]], dim=1)", "s", [pin_core.test_normalisation_sk16_model]),
    ("feed-forward residual dropped", network, "block", "return x + hdn @", "return hdn @",
     [pin_core.test_blocks_match_library_transformer_layer]),
    ("score scale 1/d_h instead of 1/sqrt(d_h)", network, "masked_attention", "/ math.sqrt(dh)", "/ dh",
     [pin_core.test_full_causal_equals_library_attention]),
    ("band one key short", network, "visibility", "(t - j <= window)", "(t - j < window)",
     [pin_core.test_one_layer_conditionals_depend_exactly_on_the_visible_sites]),
    ("prefix lost (band only)", network, "visibility", "| (j < prefix)", "| (j < 0)",
     [pin_core.test_one_layer_conditionals_depend_exactly_on_the_visible_sites]),
    ("LayerNorm without its epsilon", network, "layer_norm", "torch.sqrt(var + LN_EPS)", "torch.sqrt(var)",
     [pin_core.test_blocks_match_library_transformer_layer]),
]


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("desc,module,fname,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(desc, module, fname, old, new, pins, monkeypatch):
    monkeypatch.setattr(module, fname, mutant(module, fname, old, new))
    assert killed(pins), f"no pin catches: {desc}"


def test_muon_matrix_left_out_fails_a_pin(monkeypatch):
    monkeypatch.setattr(muon, "MATRIX_KINDS", ("qkv.w", "ffn1.w"))
    assert killed([pin_muon.test_muon_takes_exactly_the_layer_matrices])


def test_unmutated_oracle_passes_the_same_pins():
    """The harness itself: the pins used above pass on the oracle as it is."""
    pins = [p for m in MUTANTS for p in m[5]] + [pin_muon.test_muon_takes_exactly_the_layer_matrices]
    assert not killed(pins)
