"""The oracle's pins must catch plausible mistakes: each mutant below is the
oracle with one planted error (compiled on the CPU into a temporary
library); at least one pin of tests/test_oracle.py has to fail on it."""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
import test_oracle as T

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "traj.c")

# (name, original text, planted error, pins expected to notice)
MUTANTS = [
    ("kraus_scale_1_over_p", "scale(psi, n, 1.0 / sqrt(p_chosen));",
     "scale(psi, n, 1.0 / p_chosen);",
     [T.test_state_stays_normalised_through_kraus_and_measure]),
    ("cx_control_target_swapped", "case O_CX: apply_cx(psi, n, op->q[0], op->q[1]); break;",
     "case O_CX: apply_cx(psi, n, op->q[1], op->q[0]); break;",
     [T.test_gates_match_independent_dense_application]),
    ("u3_lambda_sign", "m[1] = -cexp(I * la) * s;", "m[1] = -cexp(-I * la) * s;",
     [T.test_round_trip_returns_to_zero_state, T.test_gates_match_independent_dense_application]),
    ("u3_phase_on_wrong_entry", "m[3] = cexp(I * (ph + la)) * c;", "m[3] = cexp(I * (ph - la)) * c;",
     [T.test_u3_special_cases, T.test_gates_match_independent_dense_application]),
    ("readout_rates_swapped", "double pf = bit ? ro10 : ro01;", "double pf = bit ? ro01 : ro10;",
     [T.test_readout_closed_form, T.test_readout_flip_draw]),
    ("reset_keeps_one", "if (op->kind != O_MEASURE) reset_measured(psi, n, op, o);",
     "if (op->kind == O_MEASURE_RESET && 0) reset_measured(psi, n, op, o);",
     [T.test_reset_then_measure_is_zero]),
    ("rules_in_reverse_order", "for (int r = 0; r < n_rules; ++r) {\n            if (!((rules[r]",
     "for (int r = n_rules - 1; r >= 0; --r) {\n            if (!((rules[r]",
     [T.test_oracle_sample_mismatch_detects_wrong_channel_order]),
    ("philox_wrong_multiplier", "0xCD9E8D57u * (uint64_t)c2", "0xCD9E8D59u * (uint64_t)c2",
     [T.test_philox_known_answers]),
    ("uniform_drops_a_bit", "uint64_t lo = x[1] >> 6; /* 26 bits */", "uint64_t lo = x[1] >> 7; /* 26 bits */",
     [T.test_uniform_is_53bit_from_first_two_words]),
    ("pauli_first_term_skipped", "for (int j = 0; j < ru->n_terms; ++j) {\n        run += ru->prob[j];",
     "for (int j = 1; j < ru->n_terms; ++j) {\n        run += ru->prob[j];",
     [T.test_table1_bitflip_follows_cumulative_threshold, T.test_depolarizing_closed_form]),
    ("kraus_compare_reversed", "if (u * N < run) { chosen = j; p_chosen = p; break; }",
     "if (u * N > run) { chosen = j; p_chosen = p; break; }",
     [T.test_kraus_choice_follows_running_sum, T.test_amplitude_damping_closed_form]),
    ("measure_bit_order_reversed", "for (int t = 0; t < m; ++t) pat |= ((i >> op->q[t]) & 1ull) << t;\n        P[pat]",
     "for (int t = 0; t < m; ++t) pat |= ((i >> op->q[m - 1 - t]) & 1ull) << t;\n        P[pat]",
     [T.test_dm_equals_tree_and_oracle_samples]),
    ("condition_ignored", "if (op->cmask && (creg & op->cmask) != op->cval) continue;",
     "if (0 && op->cmask && (creg & op->cmask) != op->cval) continue;",
     [T.test_feed_forward_conditional_closed_form, T.test_conditionals_dm_equals_tree_and_oracle_samples]),
    ("branch_op_inverted", "const uint64_t bit = (creg & op->cmask) == op->cval;",
     "const uint64_t bit = (creg & op->cmask) != op->cval;",
     [T.test_branch_op_sets_bit_from_register]),
]


def _build_mutant(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutant {name}: anchor not found once"
    path_c = os.path.join(tmp, f"{name}.c")
    with open(path_c, "w") as fh:
        fh.write(src.replace(old, new))
    lib = os.path.join(tmp, f"lib_{name}.so")
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                           "-o", lib, path_c, "-lm"])
    return lib


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, pins, monkeypatch):
    tmp = tempfile.mkdtemp(prefix="oracle_mutant_")
    try:
        lib = _build_mutant(tmp, name, old, new)
        monkeypatch.setattr(oracle, "_LIB_PATH", lib)
        monkeypatch.setattr(oracle, "_lib", None)
        caught = []
        for pin in pins:
            kwargs = {"seed": 0} if "seed" in pin.__code__.co_varnames[:pin.__code__.co_argcount] else {}
            try:
                pin(**kwargs)
            except AssertionError:
                caught.append(pin.__name__)
        assert caught, f"no pin noticed mutant {name}"
    finally:
        monkeypatch.setattr(oracle, "_lib", None)
        shutil.rmtree(tmp, ignore_errors=True)


def test_unmutated_oracle_passes_the_same_pins():
    for _, _, _, pins in MUTANTS:
        for pin in pins:
            kwargs = {"seed": 0} if "seed" in pin.__code__.co_varnames[:pin.__code__.co_argcount] else {}
            pin(**kwargs)
