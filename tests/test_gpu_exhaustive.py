"""Every program of length 6 over 2 variables, checked on the GPU and compared byte for
byte with the oracle.

The alphabet of one statement is 5 effects x 2 sides x 2 variables = 20 symbols, so there
are 20^6 = 64,000,000 programs.  Every shorter program is a prefix of a length-6 one and a
statement's outputs depend only on the statements before it, so this also covers every
program of length <= 6.  Programs are packed into traces of up to 2^21 programs with
disjoint variables (program q owns ids 2q and 2q + 1, every id starts at (V,I)), and the
statements are interleaved: the trace holds statement 0 of every program, then statement 1
of every program, and so on, so that each variable's events lie in different tiles and the
carries between tiles are exercised on every program."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

LENGTH = 6
SYMBOLS = 20
N_PROGRAMS = SYMBOLS ** LENGTH
PER_TRACE = 1 << 21


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def programs_trace(p0: int, m: int) -> np.ndarray:
    """Events of programs p0 .. p0+m-1, statement-major.  Statement j of program p is the
    j-th base-20 digit s of p: variable s % 2, effect (s // 2) % 5 (r, w, Push, Pull, Noop),
    side s // 10."""
    p = np.arange(p0, p0 + m, dtype=np.int64)
    q = np.arange(m, dtype=np.uint32)
    out = np.empty(LENGTH * m, np.uint32)
    for j in range(LENGTH):
        s = (p // SYMBOLS ** j) % SYMBOLS
        var = (s % 2).astype(np.uint32)
        op = ((s // 2) % 5).astype(np.uint32)
        side = (s // 10).astype(np.uint32)
        out[j * m:(j + 1) * m] = (2 * q + var) | (op << np.uint32(24)) | (side << np.uint32(27))
    return out


def test_program_packing_is_a_bijection():
    """The packing enumerates each program exactly once (checked on the first and the last
    traces: every (program, statement) symbol appears, and distinct programs differ)."""
    m = 4096
    for p0 in (0, N_PROGRAMS - m):
        e = programs_trace(p0, m).reshape(LENGTH, m)
        sym = ((e >> 27) & 1) * 10 + ((e >> 24) & 7) * 2 + (e & 1)
        code = sum(sym[j].astype(np.int64) * SYMBOLS ** j for j in range(LENGTH))
        assert np.array_equal(code, np.arange(p0, p0 + m))


@pytest.fixture(scope="module")
def ctx():
    from paper_1910_11110_amd import vcheck as V
    c = V.Context(0)
    yield c
    c.close()


@pytest.mark.gpu
def test_every_program_of_length_6_over_2_variables(ctx):
    from paper_1910_11110_amd import vcheck as V
    done = 0
    k = 0
    while done < N_PROGRAMS:
        m = min(PER_TRACE, N_PROGRAMS - done)
        e = programs_trace(done, m)
        say(f"[exhaustive] trace {k}: programs {done} .. {done + m - 1} ({e.size} events, {2 * m} ids)")
        t = V.Trace.load(ctx, e, 2 * m)
        t.check()
        ctx.sync()
        st, fin, viol = t.status(), t.final(), t.violations()
        t.free()
        ref = O.check(e, 2 * m)
        if not np.array_equal(st, ref.status):
            bad = np.nonzero(st != ref.status)[0]
            i = int(bad[0])
            raise AssertionError(f"{bad.size} status bytes differ; first at event {i} (program {done + i % m}, "
                                 f"statement {i // m}): gpu {st[i]:#x} oracle {ref.status[i]:#x}")
        assert np.array_equal(fin, ref.final), "final statuses differ"
        assert viol.total == ref.violations.size and np.array_equal(viol.indices, ref.violations)
        assert viol.first == ref.first
        # Property Safety on the GPU's bytes: from (V,I) no status is ever (I,I)
        assert not ((st & 3) == 0).any() and not (((st >> 2) & 3) == 0).any()
        done += m
        k += 1
    assert done == N_PROGRAMS
