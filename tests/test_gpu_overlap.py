"""Parity of the overlapping-array path (interval sweep + expansion + check) with the oracle."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen
from tests.helpers import load_yaml

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


def run(ctx, events, lo, hi, init=None):
    from paper_1910_11110_amd import vcheck as V
    t = V.Trace.load(ctx, events, lo.size, init)
    t.set_arrays(lo, hi)
    return t


def assert_overlap(ctx, events, lo, hi, init=None, label=""):
    say(f"[overlap] {label} n={events.size} arrays={lo.size}")
    t = run(ctx, events, lo, hi, init)
    off, nbr = t.overlap_sets()
    roff, rnbr = O.overlap_sets(lo, hi)
    assert np.array_equal(off, roff) and np.array_equal(nbr, rnbr), f"{label}: overlap sets differ"
    t.check()
    ctx.sync()
    ref = O.check_overlap(events, lo, hi, init, sets=(roff, rnbr))
    st = t.status()
    if not np.array_equal(st, ref.status):
        bad = np.nonzero(st != ref.status)[0]
        raise AssertionError(f"{label}: {bad.size} statuses differ, first {bad[0]}")
    assert np.array_equal(t.final(), ref.final), f"{label}: final differs"
    v = t.violations()
    assert v.total == ref.violations.size and np.array_equal(v.indices, ref.violations) and v.first == ref.first
    assert t.induced_stuck() == ref.n_induced_stuck
    t.free()
    return ref


def test_overlap_pvector_example(ctx):
    ex = load_yaml("overlap_example.yaml")
    names = list(ex["arrays"])
    lo = np.array([ex["arrays"][n][0] for n in names], np.uint32)
    hi = np.array([ex["arrays"][n][1] for n in names], np.uint32)
    e = gen.plain_events(2000, len(names), 1)
    assert_overlap(ctx, e, lo, hi, label="pvector")


@pytest.mark.parametrize("n_arr,space,maxlen,n", [(1, 16, 4, 100), (50, 256, 64, 5000), (2000, 1 << 16, 512, 100_000),
                                                  (20_000, 1 << 20, 4096, 1_000_003)])
def test_overlap_shapes(ctx, n_arr, space, maxlen, n):
    lo, hi = gen.intervals(n_arr, n_arr + 3, space=space, max_len=maxlen)
    e = gen.plain_events(n, n_arr, n_arr + 4)
    assert_overlap(ctx, e, lo, hi, label=f"{n_arr} arrays")


def test_overlap_identical_and_nested_intervals(ctx):
    lo = np.array([0, 0, 2, 5, 5, 100], np.uint32)
    hi = np.array([10, 10, 3, 6, 6, 101], np.uint32)
    e = gen.plain_events(20_000, 6, 12)
    assert_overlap(ctx, e, lo, hi, label="identical/nested")


def test_overlap_unsafe_initial_statuses(ctx):
    """Arrays starting at (I,I): induced acquisitions get stuck and are counted."""
    lo, hi = gen.intervals(500, 13, space=1 << 14, max_len=256)
    init = gen.below(gen.draws(13, 300, 0, 500), 4).astype(np.uint8)
    e = gen.plain_events(50_000, 500, 13)
    ref = assert_overlap(ctx, e, lo, hi, init=init, label="init (I,I)")
    assert ref.n_induced_stuck > 0


def test_overlap_workload_full_size(ctx):
    """The overlapping-array workload: 2^16 intervals in 2^24 addresses, 2^24 events."""
    lo, hi = gen.intervals(1 << 16, 0)
    e = gen.plain_events(1 << 24, 1 << 16, 0)
    assert_overlap(ctx, e, lo, hi, label="full 2^16 x 2^24")


@pytest.mark.parametrize("n,n_arr,space,maxlen", [(1, 1, 64, 8), (4097, 50, 1024, 64), (300_001, 4000, 1 << 18, 512),
                                                  (2_000_003, 1 << 16, 1 << 24, 4096)])
def test_bucket_and_general_overlap_paths_agree(n, n_arr, space, maxlen):
    """The bucket-engine route (the combined stream as 32-bit words) and the general sorted
    route give identical bytes, violations and stuck induced counts, also from initial
    (I,I) statuses, where induced acquisitions get stuck."""
    import os

    from paper_1910_11110_amd import vcheck as V
    lo, hi = gen.intervals(n_arr, n + 1, space=space, max_len=maxlen)
    e = gen.plain_events(n, n_arr, n + 2)
    init = (np.arange(n_arr) % 4).astype(np.uint8)
    outs = []
    for general in (False, True):
        if general:
            os.environ["VC_GENERAL_PATH"] = "1"
        try:
            c = V.Context(0)
            t = V.Trace.load(c, e, n_arr, init)
            t.set_arrays(lo, hi)
            t.check()
            c.sync()
            v = t.violations()
            outs.append((t.status(), t.final(), v.indices, v.first, t.induced_stuck()))
            t.free()
            c.close()
        finally:
            os.environ.pop("VC_GENERAL_PATH", None)
    a, b = outs
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert a[3] == b[3] and a[4] == b[4]
    ref = O.check_overlap(e, lo, hi, init)
    assert np.array_equal(a[0], ref.status) and a[4] == ref.n_induced_stuck


def test_overlap_dense_overlaps(ctx):
    """Every array overlaps most others (300 arrays of 300-700 elements in 1,000
    addresses): a write induces hundreds of items, so one event's items span several
    steps of the expansion's 64-item walk."""
    rng = np.random.default_rng(5)
    lo = rng.integers(0, 500, 300).astype(np.uint32)
    hi = (lo + rng.integers(300, 500, 300)).astype(np.uint32)
    e = gen.plain_events(20_000, 300, 14)
    assert_overlap(ctx, e, lo, hi, label="dense overlaps")
