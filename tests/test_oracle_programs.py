"""Pins of the oracle's interpreter of structured programs (Section 3.2; Figure
"Operational semantics of validity status"): random programs against the small-step
rules taken literally, straight-line programs against the plain check, the translation
of access modes written with its If statements, While against its unrolling, and
choice conditions."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen
from tests import pin_models as PM


def run(stmts, n_vars, choice=0, init=None, fuel=1 << 12):
    w = np.array(gen.program_words(stmts), np.uint32)
    return O.run_programs(np.array([0, w.size], np.uint64), w, n_vars, np.array([choice], np.uint64),
                          None if init is None else np.array(init, np.uint8), fuel)


@pytest.mark.parametrize("seed", range(4))
def test_random_programs_follow_the_small_step_rules(seed):
    rng = np.random.default_rng(seed)
    for trial in range(300):
        n_vars = int(rng.integers(1, 4))
        prog = gen.random_program(rng, n_vars, int(rng.integers(1, 24)))
        init = [int(rng.integers(1, 4)) for _ in range(n_vars)]
        choice = int(rng.integers(0, 1 << 63))
        fuel = int(rng.integers(1, 200))
        r = run(prog, n_vars, choice, init, fuel)
        steps, effects, stuck_at, done, store = PM.structured_run(
            prog, {v: PM.str_of(init[v]) for v in range(n_vars)}, choice, fuel)
        if stuck_at is not None:          # halted: the oracle flags the same effect first
            assert r.stuck[0] > 0 and r.first[0] == stuck_at, (trial, prog)
        else:
            assert r.stuck[0] == 0 and bool(r.done[0]) == done and r.steps[0] == steps, (trial, prog)
            assert r.effects[0] == effects
            assert [PM.str_of(int(c)) for c in r.final[0]] == [store[v] for v in range(n_vars)]


def test_straight_line_programs_are_the_plain_check():
    e = gen.plain_events(3000, 6, 4)
    stmts = [("E", int((w >> 24) & 7), int((w >> 27) & 1), int(w & 0xFFFFFF)) for w in e]
    r = run(stmts, 6, fuel=1 << 20)
    ref = O.check(e, 6)
    assert r.done[0] and r.effects[0] == 3000 and r.steps[0] == 3000
    assert np.array_equal(r.final[0], ref.final) and r.stuck[0] == ref.violations.size and r.first[0] == ref.first


def test_translation_with_its_if_statements():
    """Figure "Semantics of access modes and programs": [[R x#]] is an If on isValid x#
    (remIsValid on the GPU) whose else-branch transfers x and x#; written as structured
    programs (Noop being the empty sequence), the statuses equal the fixed-arity
    translation's."""
    for seed in range(3):
        ct = gen.component_trace(300, 6, seed, kmax=4)
        nv = ct.n_vars
        stmts = []
        for c in range(ct.n_comp):
            ds = ct.decls[int(ct.comp_off[c]):int(ct.comp_off[c + 1])]
            for d in ds:
                v, mode, side = int(d & 0xFFFFFF), int((d >> 24) & 3), int((d >> 27) & 1)
                if mode in (0, 2):
                    t = 3 if side == 0 else 2  # local Pull (CPU) / local Push (GPU)
                    stmts.append(("I", (side, nv + v), [], [("E", t, 0, v), ("E", t, 0, nv + v)]))
                if mode in (1, 2):
                    stmts.append(("E", 1, side, nv + v))
            for d in ds:
                v, mode, side = int(d & 0xFFFFFF), int((d >> 24) & 3), int((d >> 27) & 1)
                if mode in (0, 2):
                    stmts.append(("E", 0, side, v))
                if mode in (1, 2):
                    stmts.append(("E", 1, side, v))
        r = run(stmts, 2 * nv, fuel=1 << 20)
        ref = O.check(O.translate(ct.comp_off, ct.decls, nv), 2 * nv)
        assert r.done[0] and np.array_equal(r.final[0], ref.final) and r.stuck[0] == ref.violations.size == 0


def test_while_equals_its_unrolling():
    rng = np.random.default_rng(5)
    for trial in range(200):
        body = gen.random_program(rng, 2, int(rng.integers(1, 10)), depth=2)
        cond = (int(rng.integers(3)), int(rng.integers(2)))
        rest = gen.random_program(rng, 2, 4, depth=3)
        choice = int(rng.integers(0, 1 << 63))
        a = run([("W", cond, body)] + rest, 2, choice, [1, 2], 500)
        b = run([("I", cond, body + [("W", cond, body)], [])] + rest, 2, choice, [1, 2], 500)
        for f in ("steps", "effects", "stuck", "first", "done", "final"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), (trial, f)


def test_choice_conditions_and_fuel():
    # While(choice) { r x }: the first evaluations give 1, 1, 1, then 0
    r = run([("W", (2, 0), [("E", 0, 0, 0)])], 1, choice=0b0111)
    assert r.done[0] and r.steps[0] == 4 + 3 and r.effects[0] == 3
    # While(isValid x) { w GPU x }: one iteration, x ends on the GPU only
    r = run([("W", (0, 0), [("E", 1, 1, 0)])], 1)
    assert r.done[0] and r.steps[0] == 3 and r.final[0][0] == 2
    # While(isValid x) { r x } never ends: the fuel stops it
    r = run([("W", (0, 0), [("E", 0, 0, 0)])], 1, fuel=101)
    assert not r.done[0] and r.steps[0] == 101 and r.effects[0] == 50


def test_malformed_programs():
    for words in ([(1 << 30) | 0, 5, 0], [(3 << 30)], [(2 << 30) | (3 << 24)], [5 | (6 << 24)], [(1 << 30) | 9, 0]):
        w = np.array(words, np.uint32)
        with pytest.raises(O.OracleError):
            O.run_programs(np.array([0, w.size], np.uint64), w, 2)
