"""Parity of the structured-program interpreter (HIP path through the C ABI) with the
oracle: reductions, effects, stuck effects, the first stuck effect, completion and the
final statuses of every program."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1910_11110_amd import vcheck as V
    c = V.Context(0)
    yield c
    c.close()


def assert_parity(ctx, P, fuel, label=""):
    from paper_1910_11110_amd import vcheck as V
    say(f"[programs] {label}: {P.prog_off.size - 1} programs, {P.words.size} words, fuel {fuel}")
    g = V.Programs(ctx, P.prog_off, P.words, P.n_vars, P.choice, P.init, fuel)
    got = g.read()
    g.free()
    ref = O.run_programs(P.prog_off, P.words, P.n_vars, P.choice, P.init, fuel)
    names = ["steps", "effects", "stuck", "first", "done", "final"]
    for name, a, b in zip(names, got, (ref.steps, ref.effects, ref.stuck, ref.first, ref.done, ref.final)):
        if not np.array_equal(a, b):
            i = int(np.nonzero((a != b).reshape(a.shape[0], -1).any(axis=1))[0][0])
            raise AssertionError(f"{label}: {name} differs first at program {i}: gpu {a[i]} oracle {b[i]}")


@pytest.mark.parametrize("n_prog,n_vars,fuel,max_words", [(1, 1, 1, 8), (129, 3, 50, 16), (5000, 8, 1000, 48),
                                                          (40_001, 64, 300, 64), (100_003, 17, 4096, 64)])
def test_programs_shapes(ctx, n_prog, n_vars, fuel, max_words):
    P = gen.structured_programs(n_prog, n_vars, n_prog + n_vars, n_templates=min(512, n_prog), max_words=max_words)
    assert_parity(ctx, P, fuel, label=f"{n_prog} programs")


def test_programs_empty_and_deep(ctx):
    """An empty program, and While / If nested 16 deep (the limit)."""
    stmts = [("E", 1, 1, 0)]
    for d in range(15):
        stmts = [("W", (1, 0), stmts + [("E", 1, 0, 0)])] if d % 2 else [("I", (2, 0), stmts, [("E", 0, 1, 0)])]
    w = np.array(gen.program_words(stmts), np.uint32)
    P = gen.Programs(np.array([0, 0, w.size], np.uint64), w, 1, np.array([5, 0x5555], np.uint64), None)
    assert_parity(ctx, P, 10_000, label="empty and deep")


def test_programs_malformed(ctx):
    from paper_1910_11110_amd import vcheck as V
    stmts = [("E", 1, 1, 0)]
    for _ in range(17):
        stmts = [("I", (0, 0), stmts, [])]
    w = np.array(gen.program_words(stmts), np.uint32)
    with pytest.raises(O.OracleError) as want:
        O.run_programs(np.array([0, w.size], np.uint64), w, 1)
    with pytest.raises(V.VCError) as got:
        V.Programs(ctx, np.array([0, w.size], np.uint64), w, 1)
    assert got.value.code == V.VC_EINVAL and str(want.value) in str(got.value)


@pytest.mark.timeout(600)
def test_programs_workload_full_size(ctx):
    """The measured workload: 2^20 programs over 16 variables from 4,096 templates, fuel 4096."""
    say("[programs] generating the full-size workload")
    P = gen.structured_programs(1 << 20, 16, 0)
    assert_parity(ctx, P, 1 << 12, label="full size")
