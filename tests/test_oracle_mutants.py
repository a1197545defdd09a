"""The pins must catch plausible mistakes in the oracle.

Each case below plants one mistake (a non-strict comparison, a transposed
operand, a dropped term, a wrong sign, a wrong index or constant) in a copy of
oracle/oracle.c, builds it with gcc into a temporary directory, routes the
oracle wrappers through it, and checks that at least one pin of
test_oracle_pins fails.  CPU only; nothing here touches the product path.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

MUTANTS = {
    "non-strict feasibility": ("if (!(lat[x] < target[i * n_hw + h]))",
                               "if (!(lat[x] <= target[i * n_hw + h]))"),
    "cost tie to highest index": ("return lhs < rhs;", "return lhs <= rhs;"),
    "transposed batch operand": ("(__int128)cost[x] * (__int128)batch[y]",
                                 "(__int128)cost[x] * (__int128)batch[x]"),
    "max instead of sum along path": ("int64_t nv = ref_lat[v] + m;",
                                      "int64_t nv = ref_lat[v] > m ? ref_lat[v] : m;"),
    "shortest instead of longest path": ("if (c > m)", "if (m == 0 || c < m)"),
    "queueing time added": ("(__int128)slo - (__int128)elapsed - (__int128)q",
                            "(__int128)slo - (__int128)elapsed + (__int128)q"),
    "wrong Q16 scale": ("return (int64_t)(p / Q_ONE);", "return (int64_t)(p / 65535);"),
    "branch probability ignored": ("if (mode == ORACLE_PAPER)\n        return w_succ;",
                                   "if (mode >= 0)\n        return w_succ;"),
    "fallback tie to highest index": ("if (lat[x] < lat[fast])", "if (lat[x] <= lat[fast])"),
    "reference tie to highest index": ("if (best < 0 || res[x] < res[best])",
                                       "if (best < 0 || res[x] <= res[best])"),
    "reference ignores batch": ("if (hw[x] != 0 || batch[x] != 1)", "if (hw[x] != 0)"),
    "no clamp past the deadline": ("if (r < 0)\n        r = 0;", "if (r < -2147483647)\n        r = 0;"),
    "numerator uses wrong op": ("(__int128)ref_lat[v] * (__int128)R",
                                "(__int128)ref_lat[0] * (__int128)R"),
    "denominator uses wrong op": ("num / (__int128)W[v]", "num / (__int128)W[0]"),
    "slack of backend 0 for every config": ("if (!(lat[x] < target[i * n_hw + h]))",
                                            "if (!(lat[x] < target[i * n_hw]))"),
    "sweep stops one early": ("for (int32_t v = n_ops - 1; v >= 0; --v) {",
                              "for (int32_t v = n_ops - 1; v >= 1; --v) {"),
}

PIN_CHECKS = [
    pins.test_worked_example_relaxation_and_targets,
    pins.test_worked_example_select,
    lambda: pins.test_single_op_gets_whole_remaining_time(oracle.PAPER),
    lambda: pins.test_equal_reference_chain(3),
    pins.test_prob_chain_closed_form,
    pins.test_symmetric_fork_equals_one_branch,
    pins.test_random_dags_full_decision_against_brute_force,
    pins.test_select_against_exact_rationals_with_many_ties,
    pins.test_reference_rule,
    pins.test_invalid_invocations,
    lambda: pins.test_invariants("c1q"),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    with open(oracle.SRC_PATH) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site for '{name}' not unique"
    c = tmp_path / "mutant.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", str(c), "-o", str(so)])
    caught = []
    with oracle.use(str(so)):
        for check in PIN_CHECKS:
            try:
                check()
            except (AssertionError, oracle.OracleError):
                caught.append(getattr(check, "__name__", "lambda"))
    assert caught, f"no pin caught the planted mistake '{name}'"


def test_unmutated_oracle_passes_every_check():
    with oracle.use(oracle.LIB_PATH):
        for check in PIN_CHECKS:
            check()
