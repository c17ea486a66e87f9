"""The generation-control pins catch plausible mistakes in the oracle.

Each case plants one mistake in a scratch copy of the oracle's C source (a
phase moved, a tie sent to the other particle, the mutation phase shifted, the
exchange trigger inverted), builds it, and runs the pins of
``test_oracle_control.py`` against that build in a subprocess: at least the
named pin must fail. The committed oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dpso_oracle.c")

MUTANTS = {
    # the global best is taken before the mutation instead of after it
    "gbest_before_mutation": (
        "    if (prm->mutation_period > 0 && t % prm->mutation_period == 0)\n"
        "        st->n_reshuffled += or_mutation(D, prm, st, t, NULL);\n"
        "    int32_t improved = or_update_gbest(st);\n",
        "    int32_t improved = or_update_gbest(st);\n"
        "    if (prm->mutation_period > 0 && t % prm->mutation_period == 0)\n"
        "        st->n_reshuffled += or_mutation(D, prm, st, t, NULL);\n",
        "test_mutation_precedes_the_global_best_update"),
    # ties of the global best go to the highest index
    "gbest_tie_highest": (
        "        if (st->FP[p] < st->FP[g]) g = p;\n    if (st->FP[g] < st->FG) {",
        "        if (st->FP[p] <= st->FP[g]) g = p;\n    if (st->FP[g] < st->FG) {",
        "test_global_best_ties_go_to_the_lowest_index"),
    # mutation on t mod period = 1
    "mutation_phase_shifted": (
        "t % prm->mutation_period == 0)\n        st->n_reshuffled",
        "t % prm->mutation_period == 1)\n        st->n_reshuffled",
        "test_mutation_only_on_multiples_of_the_period"),
    # the exchange runs when the global best improved instead of when it did not
    "trigger_inverted": (
        "(prm->ee_trigger == EE_ON_STALL && !improved)) {",
        "(prm->ee_trigger == EE_ON_STALL && improved)) {",
        "test_on_stall_exchange_runs_when_the_global_best_does_not_improve"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(tmp_path, name):
    old, new, pin = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "the planted site no longer matches the oracle source"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                           str(mutant), "-lm"])
    env = dict(os.environ, DPSO_ORACLE_LIB=str(lib))
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_control.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True)
    assert res.returncode != 0, res.stdout[-2000:]
    assert f"FAILED tests/test_oracle_control.py::{pin}" in res.stdout, res.stdout[-2000:]
