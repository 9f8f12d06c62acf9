"""Pins of the oracle's check with partial vectors created and destroyed during the
trace (Section 4.3, "Towards an implementation in VectorPU"; appendix "Partial
Vectors"): a worked scenario, the reduction to the static overlap check when nothing
is created or destroyed, the element-level meaning of the array statuses, and the
lifetime rules."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen
from tests import pin_models as PM
from tests.helpers import PAIRS, SIDES, load_yaml

OPS = {"r": 0, "w": 1, "Push": 2, "Pull": 3, "Noop": 4, "create": 6, "destroy": 7}
NAMES = ["r", "w", "Push", "Pull", "Noop"]


def _scenario():
    ex = load_yaml("dynamic_pvectors.yaml")
    names = list(ex["arrays"])
    ids = {a: i for i, a in enumerate(names)}
    lo = np.array([ex["arrays"][a]["lo"] for a in names], np.uint32)
    hi = np.array([ex["arrays"][a]["hi"] for a in names], np.uint32)
    mo = np.array([O.NO_MOTHER if ex["arrays"][a]["mother"] is None else ids[ex["arrays"][a]["mother"]]
                   for a in names], np.uint32)
    ev = np.array([ids[a] | (OPS[op] << 24) | (SIDES[side] << 27) for op, side, a in ex["events"]], np.uint32)
    return ex, names, ids, lo, hi, mo, ev


def test_dynamic_worked_scenario():
    ex, names, ids, lo, hi, mo, ev = _scenario()
    r = O.check_dynamic(ev, lo, hi, mo)
    assert list(O.pre(r.status)) == [PAIRS[f"({s[0]},{s[1]})"] for s in ex["pre"]]
    assert list(O.post(r.status)) == [PAIRS[f"({s[0]},{s[1]})"] for s in ex["post"]]
    assert list(r.violations) == ex["stuck"] and r.first == ex["stuck"][0]
    assert r.n_induced == ex["induced"] and r.n_induced_stuck == 0
    for a, s in ex["final"].items():
        assert r.final[ids[a]] == PAIRS[f"({s[0]},{s[1]})"], a


def test_dynamic_without_lifecycle_is_the_static_overlap_check():
    """With every array live from start to end the registry never changes, and the
    check is the static overlap check (whose overlap sets are the same pair test)."""
    for seed in range(3):
        lo, hi = gen.intervals(400, seed, space=1 << 13, max_len=256)
        e = gen.plain_events(30_000, 400, seed + 10)
        a = O.check_dynamic(e, lo, hi, np.full(400, O.NO_MOTHER, np.uint32))
        b = O.check_overlap(e, lo, hi)
        assert np.array_equal(a.status, b.status) and np.array_equal(a.final, b.final)
        assert np.array_equal(a.violations, b.violations) and a.n_induced == b.n_induced


def test_dynamic_registry_list_and_overlap_sets_agree():
    """The two ways of finding the induced targets (the live list searched in full, the
    overlap sets filtered by liveness) give the same results."""
    for seed in range(3):
        d = gen.dynamic_trace(40_000, 8, 600, seed, space=1 << 14, max_len=512)
        a = O.check_dynamic(d.events, d.lo, d.hi, d.mother)
        b = O.check_dynamic(d.events, d.lo, d.hi, d.mother, sets=O.overlap_sets(d.lo, d.hi))
        assert np.array_equal(a.status, b.status) and np.array_equal(a.final, b.final)
        assert np.array_equal(a.violations, b.violations) and a.n_induced == b.n_induced > 0


def _element_replay(ev, lo, hi, mo, r):
    """Replays a dynamic trace on an element-level model (every address has its own
    status pair; an array-level r, w, Push or Pull acts on every element of the array,
    an induced RW acquires the whole array as its declaration does) and checks, after
    every event, that each live array's status is a safe abstraction of each of its
    elements (Theorem on overlapping arrays; a created partial vector inherits a status
    that abstracts its mother's elements), and that an event the oracle does not flag
    succeeds on every element."""
    n_arr = lo.size
    names = [f"a{i}" for i in range(n_arr)]
    model = PM.ElementModel(int(hi.max()), {names[i]: (int(lo[i]), int(hi[i])) for i in range(n_arr)})
    created = {int(x) for x, op in zip(ev & 0xFFFFFF, (ev >> 24) & 7) if op == 6}
    live = {i for i in range(n_arr) if i not in created}
    for i, w in enumerate(ev):
        x, op, side = int(w & 0xFFFFFF), int((w >> 24) & 7), int((w >> 27) & 1)
        if op == 6:
            live.add(x)
            model.abs[names[x]] = PM.str_of(int(O.post(r.status)[i]))
        elif op == 7:
            live.discard(x)
        else:
            # the model's abstract status (induced RW included) is the oracle's pre-status
            assert PM.code_of(model.abs[names[x]]) == int(O.pre(r.status)[i]), f"event {i}: pre-status of {x}"
            flagged = bool(O.stuck(r.status)[i])
            before = len(model.stuck)
            if not flagged:
                a, (l, h) = names[x], (int(lo[x]), int(hi[x]))
                for k in range(l, h):
                    model._elem_step(k, NAMES[op], side == 1, (NAMES[op], a, k))
                model.abs[a] = PM.str_of(int(O.post(r.status)[i]))
                assert len(model.stuck) == before, f"event {i} succeeds on the array but not on its elements"
            if op == 1:
                for y in sorted(live):
                    if y != x and lo[x] < hi[y] and lo[y] < hi[x]:
                        model.declare("RW", "GPU" if side else "CPU", names[y])
        for y in live:
            l, h = int(lo[y]), int(hi[y])
            for k in range(l, h):
                assert PM.leq(model.abs[names[y]], model.elem[k]), f"after event {i}: array {y} element {k}"
    assert [PM.code_of(model.abs[a]) for a in names] == list(r.final)


def test_dynamic_statuses_abstract_the_elements():
    for seed in range(4):
        d = gen.dynamic_trace(1500, 3, 12, seed, space=96, max_len=24)
        r = O.check_dynamic(d.events, d.lo, d.hi, d.mother)
        _element_replay(d.events, d.lo, d.hi, d.mother, r)


def test_dynamic_scenario_statuses_abstract_the_elements():
    ex, names, ids, lo, hi, mo, ev = _scenario()
    _element_replay(ev, lo, hi, mo, O.check_dynamic(ev, lo, hi, mo))


@pytest.mark.parametrize("case", ["use-before-create", "use-after-destroy", "second-create", "create-live",
                                  "destroy-dead", "mother-dead", "side-bit", "op5"])
def test_dynamic_lifetime_errors(case):
    """Events on arrays that are not live are malformed, reported at the first one."""
    lo = np.array([0, 2, 4], np.uint32)
    hi = np.array([10, 5, 8], np.uint32)
    mo = np.array([O.NO_MOTHER, 0, 0], np.uint32)
    C, D = 6 << 24, 7 << 24
    traces = {
        "use-before-create": ([1, C | 1], 0),
        "use-after-destroy": ([C | 1, D | 1, 1], 2),
        "second-create": ([C | 1, D | 1, C | 1], 2),
        "create-live": ([C | 2, 2, C | 2], 2),
        "destroy-dead": ([C | 1, D | 1, D | 1], 2),
        "mother-dead": ([D | 0, C | 1], 1),
        "side-bit": ([C | 1 | (1 << 27)], 0),
        "op5": ([(5 << 24) | 0], 0),
    }
    ev, at = traces[case]
    with pytest.raises(O.OracleError) as e:
        O.check_dynamic(np.array(ev, np.uint32), lo, hi, mo)
    assert f"index {at}" in str(e.value)


def test_dynamic_layout_errors():
    lo = np.array([0, 2, 12], np.uint32)
    hi = np.array([10, 5, 14], np.uint32)
    for mo in ([O.NO_MOTHER, 2, O.NO_MOTHER],   # pv outside its mother
               [1, O.NO_MOTHER, O.NO_MOTHER],   # a vector inside a pvector's range
               [O.NO_MOTHER, 1, O.NO_MOTHER]):  # its own mother
        with pytest.raises(O.OracleError):
            O.check_dynamic(np.zeros(0, np.uint32), lo, hi, np.array(mo, np.uint32))
