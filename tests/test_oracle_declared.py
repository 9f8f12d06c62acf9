"""Pins of the oracle's well-declaredness check (Definitions "Well-declared program",
Section 3.4, and "Well-declared program with array access", Section 3.5; the naive rule
for overlapping arrays, Section 4.1): the paper's array example and hand-worked cases,
Theorem "Progress for well-declared programs" (a program the check accepts runs
without a stuck step), and the theorem on overlapping arrays (declarations extended by
O(M) make the naive rule hold)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen
from tests.helpers import MODES, OPS, SIDES, load_yaml

BITS = {"transfer": O.WD_TRANSFER, "read": O.WD_READ, "write": O.WD_WRITE, "unwritten": O.WD_UNWRITTEN,
        "overlap": O.WD_OVERLAP}


def _case(ex):
    names = list(ex["arrays"])
    ids = {a: i for i, a in enumerate(names)}
    lo = np.array([ex["arrays"][a][0] for a in names], np.uint32)
    hi = np.array([ex["arrays"][a][1] for a in names], np.uint32)
    decls = np.array([ids[d.split()[2]] | (MODES[d.split()[0]] << 24) | (SIDES[d.split()[1]] << 27)
                      for d in ex["decls"]], np.uint32)
    body, idx = [], []
    for b in ex["body"]:
        op, side, a, i = b.split()
        body.append(ids[a] | (OPS[op] << 24) | (SIDES[side] << 27))
        idx.append(int(i))
    return (np.array([0, decls.size], np.uint64), decls, len(names), np.array([0, len(body)], np.uint64),
            np.array(body, np.uint32), np.array(idx, np.uint32), lo, hi)


@pytest.mark.parametrize("ex", load_yaml("declared_examples.yaml"), ids=lambda e: e["name"])
def test_declared_examples(ex):
    v = O.check_declared(*_case(ex))
    want = sum(BITS[b] for b in ex["verdict"])
    assert int(v[0]) == (want | (O.WD_ILL if want else 0)), ex["name"]


def _subprogram(p, keep):
    """The components `keep` of a scalar program, as a program of their own."""
    co, bo = p.comp_off.astype(np.int64), p.body_off.astype(np.int64)
    decls = np.concatenate([p.decls[co[c]:co[c + 1]] for c in keep]) if keep.size else np.zeros(0, np.uint32)
    body = np.concatenate([p.body[bo[c]:bo[c + 1]] for c in keep]) if keep.size else np.zeros(0, np.uint32)
    nco = np.zeros(keep.size + 1, np.uint64)
    nco[1:] = np.cumsum(co[keep + 1] - co[keep])
    nbo = np.zeros(keep.size + 1, np.uint64)
    nbo[1:] = np.cumsum(bo[keep + 1] - bo[keep])
    return nco, decls, nbo, body


@pytest.mark.parametrize("seed", range(3))
def test_accepted_programs_run_without_a_stuck_step(seed):
    """Theorem "Progress for well-declared programs": keep the components the check
    accepts; their program, translated (Figure "Semantics of access modes and programs")
    and run, never gets stuck.  The components it rejects include every altered one."""
    p = gen.declared_program(30_000, 500, seed, arrays=False, p_err=0.2)
    v = O.check_declared(p.comp_off, p.decls, p.n_vars, p.body_off, p.body)
    keep = np.nonzero(v == 0)[0]
    assert 0 < keep.size < v.size
    co, de, bo, bd = _subprogram(p, keep)
    tr = O.translate(co, de, p.n_vars, bo, bd)
    assert O.check(tr, 2 * p.n_vars).violations.size == 0
    # and the rejected components, run on their own, do get stuck somewhere
    bad = np.nonzero(v != 0)[0]
    co, de, bo, bd = _subprogram(p, bad)
    assert O.check(O.translate(co, de, p.n_vars, bo, bd), 2 * p.n_vars).violations.size > 0


def test_unaltered_programs_are_well_declared():
    p = gen.declared_program(20_000, 300, 7, arrays=False, p_err=0.0)
    assert (O.check_declared(p.comp_off, p.decls, p.n_vars, p.body_off, p.body) == 0).all()


@pytest.mark.parametrize("seed", range(3))
def test_extension_makes_the_naive_overlap_rule_hold(seed):
    """Theorem on overlapping arrays (Section 4.2): a program well-declared without
    regard to overlaps, with every component's declarations extended to O(M), meets the
    naive rule of Section 4.1 as well; without the extension the rule fails."""
    p = gen.declared_program(20_000, 2000, seed, arrays=True, space=1 << 15, max_len=32, p_err=0.0)
    v0 = O.check_declared(p.comp_off, p.decls, p.n_vars, p.body_off, p.body, p.idx, p.lo, p.hi)
    assert ((v0 & ~np.uint8(O.WD_OVERLAP | O.WD_ILL)) == 0).all()
    assert (v0 & O.WD_OVERLAP).any()
    v1 = O.check_declared(p.comp_off, p.decls, p.n_vars, p.body_off, p.body, p.idx, p.lo, p.hi, extend=True)
    assert (v1 == 0).all()


def test_overlap_sets_lookup_agrees():
    """Looking the overlapping arrays up in the overlap sets gives the same verdicts as
    scanning every array."""
    for seed in range(2):
        p = gen.declared_program(6000, 1500, seed, arrays=True, space=1 << 14, max_len=32, p_err=0.1)
        sets = O.overlap_sets(p.lo, p.hi)
        for ext in (False, True):
            a = O.check_declared(p.comp_off, p.decls, p.n_vars, p.body_off, p.body, p.idx, p.lo, p.hi, ext)
            b = O.check_declared(p.comp_off, p.decls, p.n_vars, p.body_off, p.body, p.idx, p.lo, p.hi, ext, sets)
            assert np.array_equal(a, b) and (ext or (a & O.WD_OVERLAP).any())


def test_malformed_inputs():
    co = np.array([0, 2], np.uint64)
    with pytest.raises(O.OracleError, match="declaration at index 1"):
        O.check_declared(co, np.array([3, 3 | (1 << 24)], np.uint32), 8, np.array([0, 0], np.uint64),
                         np.zeros(0, np.uint32))
    with pytest.raises(O.OracleError, match="body word at index 1"):
        O.check_declared(co, np.array([3, 4], np.uint32), 8, np.array([0, 2], np.uint64),
                         np.array([3, 9], np.uint32))
    lo, hi = np.array([0, 4], np.uint32), np.array([4, 8], np.uint32)
    with pytest.raises(O.OracleError, match="body word at index 0"):
        O.check_declared(np.array([0, 1], np.uint64), np.array([0], np.uint32), 2, np.array([0, 1], np.uint64),
                         np.array([0], np.uint32), np.array([4], np.uint32), lo, hi)
