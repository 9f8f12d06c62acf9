"""The pins are strong enough: a plausible mistake planted in a copy of the oracle (on
the CPU) makes at least one pin fail.  Each mutant is a one-line edit of the C source."""
import os
import subprocess
import tempfile

import pytest

from oracle import oracle as O
from tests import test_oracle_dynamic as D
from tests import test_oracle_pins as T
from tests import test_oracle_spaces as K
from tests import test_oracle_declared as W
from tests import test_oracle_programs as G
from tests.helpers import load_yaml

MUTANTS = {
    "push-output-keeps-remote": ("/* Push : (V,X) -> (V,V) */ { { TV, TX }, { TV, TV } }",
                                 "/* Push : (V,X) -> (V,V) */ { { TV, TX }, { TV, TX } }"),
    "pull-pattern-transposed": ("/* Pull : (X,V) -> (V,V) */ { { TX, TV }, { TV, TV } }",
                                "/* Pull : (X,V) -> (V,V) */ { { TV, TX }, { TV, TV } }"),
    "w-invalidates-local": ("/* w    : (X,Y) -> (V,I) */ { { TX, TY }, { TV, TI } }",
                            "/* w    : (X,Y) -> (V,I) */ { { TX, TY }, { TI, TV } }"),
    "remote-no-swap-back": ("    if (side)\n        r = swap(r);\n", "\n"),
    "remote-no-swap": ("    if (side)\n        s = swap(s);\n", "\n"),
    "stuck-not-flagged": ("        *stuck = 1;\n        return pre;", "        *stuck = 0;\n        return pre;"),
    "initial-store-valid-both": ("sigma[v] = init ? init[v] : 1;", "sigma[v] = init ? init[v] : 3;"),
    "translate-transfer-on-decl-side": ("emit(&em, v, t, 0);", "emit(&em, v, t, (int)side);"),
    "translate-guard-on-real-var": ("int cond = side ? rem_is_valid(em.sigma[abs_v]) : is_valid(em.sigma[abs_v]);",
                                    "int cond = side ? rem_is_valid(em.sigma[v]) : is_valid(em.sigma[v]);"),
    "translate-guard-sides-swapped": ("int cond = side ? rem_is_valid(em.sigma[abs_v]) : is_valid(em.sigma[abs_v]);",
                                      "int cond = side ? is_valid(em.sigma[abs_v]) : rem_is_valid(em.sigma[abs_v]);"),
    "translate-no-abstract-write": ("emit(&em, abs_v, OP_W, (int)side);", "emit(&em, abs_v, OP_NOOP, (int)side);"),
    "overlap-rule3-ignores-premise": ("if (!(j >= 0 && ((m[j] >> 24) & 3u) == 1))", "if (1)"),
    "overlap-rw-not-inferred": ("if (mode == 2) /* RW x# */\n                    need_rw = 1;", "\n"),
    "induced-rw-wrong-side": ("cur = apply_effect(OP_W, side, cur, &st2);", "cur = apply_effect(OP_W, !side, cur, &st2);"),
    "repeated-variable-accepted": ("if ((decls[e] & 0xFFFFFFu) == v) {", "if (0) {"),
    "dynamic-inherits-initial": ("sigma[x] = mother[x] != NO_MOTHER ? sigma[mother[x]] : (init ? init[x] : 1);",
                                 "sigma[x] = init ? init[x] : 1;"),
    "dynamic-registry-keeps-destroyed": ("uint32_t last = list[--n_live]; /* remove x from the registry */\n"
                                         "            list[where[x]] = last;\n            where[last] = where[x];",
                                         ""),
    "dynamic-registry-misses-created": ("created[x] = 1;\n            where[x] = n_live;\n            list[n_live++] = x;",
                                        "created[x] = 1;"),
    "dynamic-induced-ignores-liveness": ("for (uint32_t k = 0; k < n_live; k++) {\n                uint32_t y = list[k];",
                                         "for (uint32_t k = 0; k < n_arrays; k++) {\n                uint32_t y = k;"),
    "spaces-copy-misses-target": ("        s.out[b] = KT_V;\n", ""),
    "spaces-write-keeps-others": ("s.out[j] = j == a ? KT_V : KT_I;", "s.out[j] = j == a ? KT_V : KT_X0 + j;"),
    "spaces-read-at-location-0": ("        s.in[a] = KT_V;\n        s.out[a] = KT_V;\n    } else if (op == 1)",
                                  "        s.in[0] = KT_V;\n        s.out[0] = KT_V;\n    } else if (op == 1)"),
    "declared-ignores-side": ("if ((set[i] & 0xFFFFFFu) == x && ((set[i] >> 27) & 1u) == side)",
                              "if ((set[i] & 0xFFFFFFu) == x)"),
    "declared-obligation-any-side": ("((e >> 24) & 7u) == OP_W && ((e >> 27) & 1u) == side)",
                                     "((e >> 24) & 7u) == OP_W)"),
    "declared-naive-rule-inclusive": ("if (y == x || !(lo[y] <= addr && addr < hi[y]))",
                                      "if (y == x || !(lo[y] <= addr && addr <= hi[y]))"),
    "declared-rw-not-for-writes": ("if (op == OP_W && !(mode == 1 || mode == 2))", "if (op == OP_W && !(mode == 1))"),
    "declared-transfer-allowed": ("            if (op == OP_PUSH || op == OP_PULL)\n                v8 |= 1;", ""),
    "programs-while-runs-once": ("                if (run_seq(r, pc + 2, pc + 2 + n) < 0)\n                    return -1;\n            }",
                                 "                if (run_seq(r, pc + 2, pc + 2 + n) < 0)\n                    return -1;\n"
                                 "                break;\n            }"),
    "programs-if-branches-swapped": ("if (run_seq(r, c ? pc + 3 : pc + 3 + n, c ? pc + 3 + n : pc + 3 + n + m) < 0)",
                                     "if (run_seq(r, !c ? pc + 3 : pc + 3 + n, !c ? pc + 3 + n : pc + 3 + n + m) < 0)"),
    "programs-remvalid-reads-local": ("    if (kind == 1)\n        return rem_is_valid(r->sigma[x]);",
                                      "    if (kind == 1)\n        return is_valid(r->sigma[x]);"),
    "programs-choice-bits-reversed": ("int v = (int)((r->choice >> (r->n_choice % 64)) & 1u);",
                                      "int v = (int)((r->choice >> (63 - r->n_choice % 64)) & 1u);"),
    "overlap-inclusive-upper": ("return x != y && lo[x] < hi[y] && lo[y] < hi[x];",
                                "return x != y && lo[x] <= hi[y] && lo[y] <= hi[x];"),
}


def _pins():
    T.test_effect_table_matches_printed_signatures()
    for ex in load_yaml("worked_examples.yaml"):
        T.test_worked_examples(ex)
    for ex in load_yaml("translation_examples.yaml"):
        T.test_translation_examples(ex)
    T.test_overlap_extension_pvector_example()
    T.test_safety_no_unsafe_state_from_safe_start()
    T.test_side_swap_symmetry()
    T.test_theorems_on_well_declared_component_traces(0)
    T.test_vectorpu_coherence_code_matches_abstract_status()
    T.test_overlap_write_makes_overlapping_arrays_valid_on_side_only()
    T.test_overlap_rules_keep_element_model_consistent_pvector()
    T.test_overlap_sets_brute_force_small()
    T.test_repeated_variable_in_a_component_is_rejected()
    D.test_dynamic_worked_scenario()
    D.test_dynamic_without_lifecycle_is_the_static_overlap_check()
    D.test_dynamic_statuses_abstract_the_elements()
    D.test_dynamic_scenario_statuses_abstract_the_elements()
    K.test_two_spaces_is_the_paper_calculus()
    K.test_every_program_up_to_length_3_at_k3()
    for ex in load_yaml("declared_examples.yaml"):
        W.test_declared_examples(ex)
    W.test_accepted_programs_run_without_a_stuck_step(0)
    W.test_extension_makes_the_naive_overlap_rule_hold(0)
    G.test_random_programs_follow_the_small_step_rules(0)
    G.test_straight_line_programs_are_the_plain_check()
    G.test_translation_with_its_if_statements()
    G.test_choice_conditions_and_fuel()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name):
    old, new = MUTANTS[name]
    src = open(O.SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    src = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        so = os.path.join(d, "m.so")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-O1", "-std=c99", "-w", "-fPIC", "-shared", c, "-o", so])
        saved = O._lib
        O._lib = O.load(so)
        try:
            with pytest.raises((AssertionError, O.OracleError, pytest.fail.Exception)):
                _pins()
        finally:
            O._lib = saved


def test_unmutated_oracle_passes_all_pins():
    _pins()
