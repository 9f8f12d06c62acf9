"""Pins of the oracle's check over k memory spaces (the extension to more memory
locations the paper announces in Section 3 and Section 6): the case k = 2 is the
two-space calculus, every program of length <= 3 over one variable at k = 3 agrees
with a model of valid-location sets, and relabelling the locations commutes with
the check."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen

R, W, COPY, NOOP = 0, 1, 2, 3


def kword(x, op, a=0, b=0):
    return x | (op << 24) | (a << 26) | (b << 28)


def as_spaces(events):
    """The two-space trace written with k = 2 effects: r and w at the event's side, the
    local Push / Pull as copies between locations 0 and 1 (remote ones the other way:
    Pull is rem Push)."""
    x = events & np.uint32(0xFFFFFF)
    op = (events >> np.uint32(24)) & np.uint32(7)
    side = (events >> np.uint32(27)) & np.uint32(1)
    out = np.empty_like(events)
    for i in range(events.size):
        o, s = int(op[i]), int(side[i])
        if o == 0:
            out[i] = kword(int(x[i]), R, s)
        elif o == 1:
            out[i] = kword(int(x[i]), W, s)
        elif o == 2:   # Push: from this side to the other
            out[i] = kword(int(x[i]), COPY, s, 1 - s)
        elif o == 3:   # Pull: from the other side to this one
            out[i] = kword(int(x[i]), COPY, 1 - s, s)
        else:
            out[i] = kword(int(x[i]), NOOP)
    return out


def test_two_spaces_is_the_paper_calculus():
    for seed in range(3):
        e = gen.plain_events(20_000, 37, seed)
        init = (np.arange(37) % 4).astype(np.uint8)
        a = O.check(e, 37, init)
        b = O.check_spaces(as_spaces(e), 37, 2, init)
        assert np.array_equal(b.status & 0xF, a.status & 3)
        assert np.array_equal((b.status >> 4) & 0xF, (a.status >> 2) & 3)
        assert np.array_equal(b.status >> 15, a.status >> 7)
        assert np.array_equal(b.final, a.final) and np.array_equal(b.violations, a.violations)


def set_model(program, k, start):
    """Valid-location sets: r_j needs j, w_j leaves {j}, copy a->b needs a and adds b."""
    valid, out = set(start), []
    for op, a, b in program:
        pre = frozenset(valid)
        ok = True
        if op == R:
            ok = a in valid
        elif op == W:
            valid = {a}
        elif op == COPY:
            ok = a in valid
            if ok:
                valid = valid | {b}
        out.append((pre, frozenset(valid), not ok))
    return out


def code(s):
    return sum(1 << j for j in s)


def test_every_program_up_to_length_3_at_k3():
    k = 3
    alphabet = [(R, a, 0) for a in range(k)] + [(W, a, 0) for a in range(k)] + \
        [(COPY, a, b) for a in range(k) for b in range(k)] + [(NOOP, 0, 0)]
    for length in range(1, 4):
        progs = list(itertools.product(alphabet, repeat=length))
        # every program as its own variable, all in one trace (statement-major)
        ev = np.array([kword(p, *progs[p][j]) for j in range(length) for p in range(len(progs))], np.uint32)
        for start in ({0}, {1, 2}, set()):
            init = np.full(len(progs), code(start), np.uint8)
            r = O.check_spaces(ev, len(progs), k, init)
            st = r.status.reshape(length, len(progs))
            for p, prog in enumerate(progs):
                for j, (pre, post, stuck) in enumerate(set_model(prog, k, start)):
                    got = int(st[j, p])
                    assert (got & 0xF, (got >> 4) & 0xF, got >> 15) == (code(post), code(pre), int(stuck)), \
                        (prog, start, j)


def random_k_events(n, n_ids, k, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, n_ids, n)
    op = rng.integers(0, 4, n)
    a = rng.integers(0, k, n)
    b = np.where(op == COPY, rng.integers(0, k, n), 0)
    a = np.where(op == NOOP, 0, a)
    return (x | (op << 24) | (a << 26) | (b << 28)).astype(np.uint32)


def test_relabelling_locations_commutes():
    k = 4
    e = random_k_events(30_000, 50, k, 3)
    pi = [2, 0, 3, 1]
    op = (e >> 24) & 3
    a = (e >> 26) & 3
    b = (e >> 28) & 3
    pa = np.array(pi)[a]
    pb = np.where(op == COPY, np.array(pi)[b], 0)
    pa = np.where(op == NOOP, 0, pa)
    e2 = (e & 0xFFFFFF) | (op << 24) | (pa.astype(np.uint32) << 26) | (pb.astype(np.uint32) << 28)
    init = np.arange(50, dtype=np.uint8) % 16
    perm_code = np.array([sum(1 << pi[j] for j in range(k) if (c >> j) & 1) for c in range(16)], np.uint8)
    r1 = O.check_spaces(e, 50, k, init)
    r2 = O.check_spaces(e2.astype(np.uint32), 50, k, perm_code[init])
    assert np.array_equal(perm_code[r1.status & 0xF], r2.status & 0xF)
    assert np.array_equal(r1.status >> 15, r2.status >> 15)
    assert np.array_equal(perm_code[r1.final], r2.final)


def test_valid_copies_never_vanish_from_a_valid_start():
    """From data valid somewhere, some location stays valid (the Safety property of the
    two-space calculus, for k locations)."""
    for k in (3, 4):
        e = random_k_events(50_000, 20, k, k)
        r = O.check_spaces(e, 20, k)
        assert ((r.status & 0xF) != 0).all() and (r.final != 0).all()


@pytest.mark.parametrize("word", [kword(0, R, 3), kword(0, COPY, 0, 3), kword(0, W, 0, 1), kword(0, NOOP, 1),
                                  kword(5, R, 0), (1 << 30)])
def test_malformed_space_words(word):
    with pytest.raises(O.OracleError):
        O.check_spaces(np.array([kword(0, R, 0), word], np.uint32), 4, 3)
