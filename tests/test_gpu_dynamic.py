"""Parity of the check with partial vectors created and destroyed during the trace
(HIP path through the C ABI) with the oracle: every status byte, the final table, the
violations and the stuck induced acquisitions."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen
from tests.helpers import SIDES, load_yaml

pytestmark = pytest.mark.gpu

OPS = {"r": 0, "w": 1, "Push": 2, "Pull": 3, "Noop": 4, "create": 6, "destroy": 7}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1910_11110_amd import vcheck as V
    c = V.Context(0)
    yield c
    c.close()


def run_gpu(ctx, ev, lo, hi, mo, init=None, device=False):
    from paper_1910_11110_amd import vcheck as V
    src = ev
    if device:
        import torch
        src = torch.from_numpy(ev.view(np.int32)).cuda()
    t = V.Trace.load(ctx, src, lo.size, init, lifetimes=True)
    t.set_dynamic_arrays(lo, hi, mo)
    t.check()
    ctx.sync()
    res = (t.status(), t.final(), t.violations(), t.induced_stuck())
    t.free()
    return res


def assert_parity(ctx, ev, lo, hi, mo, init=None, label="", sets=None, device=False):
    say(f"[dynamic] {label}: n={ev.size} arrays={lo.size}")
    st, fin, viol, nis = run_gpu(ctx, ev, lo, hi, mo, init, device)
    ref = O.check_dynamic(ev, lo, hi, mo, init, sets=sets)
    if not np.array_equal(st, ref.status):
        i = int(np.nonzero(st != ref.status)[0][0])
        raise AssertionError(f"{label}: status bytes differ first at {i}: gpu {st[i]:#x} oracle {ref.status[i]:#x}")
    assert np.array_equal(fin, ref.final), f"{label}: final statuses differ"
    assert viol.total == ref.violations.size and np.array_equal(viol.indices, ref.violations), label
    assert viol.first == ref.first, label
    assert nis == ref.n_induced_stuck, label


def test_dynamic_worked_scenario(ctx):
    ex = load_yaml("dynamic_pvectors.yaml")
    names = list(ex["arrays"])
    ids = {a: i for i, a in enumerate(names)}
    lo = np.array([ex["arrays"][a]["lo"] for a in names], np.uint32)
    hi = np.array([ex["arrays"][a]["hi"] for a in names], np.uint32)
    mo = np.array([O.NO_MOTHER if ex["arrays"][a]["mother"] is None else ids[ex["arrays"][a]["mother"]]
                   for a in names], np.uint32)
    ev = np.array([ids[a] | (OPS[op] << 24) | (SIDES[side] << 27) for op, side, a in ex["events"]], np.uint32)
    assert_parity(ctx, ev, lo, hi, mo, label="worked scenario")


@pytest.mark.parametrize("n,nv,npv,space,maxlen", [(3, 1, 1, 64, 8), (257, 2, 6, 256, 32), (4097, 4, 40, 1024, 64),
                                                   (100_003, 16, 600, 1 << 14, 512),
                                                   (1_000_003, 64, 4000, 1 << 20, 4096)])
def test_dynamic_shapes(ctx, n, nv, npv, space, maxlen):
    """Single events, ragged tails, several tiles of every pass, long traces."""
    d = gen.dynamic_trace(n, nv, npv, n + nv, space=space, max_len=maxlen)
    sets = O.overlap_sets(d.lo, d.hi) if n > 200_000 else None
    assert_parity(ctx, d.events, d.lo, d.hi, d.mother, label=f"dynamic {n}", sets=sets)


def test_dynamic_initial_statuses_and_device_events(ctx):
    """Initial statuses other than (V,I) (including (I,I), whose induced acquisitions get
    stuck) and events resident on the device."""
    d = gen.dynamic_trace(200_000, 8, 300, 77, space=1 << 13, max_len=256)
    init = (np.arange(d.lo.size) % 4).astype(np.uint8)
    assert_parity(ctx, d.events, d.lo, d.hi, d.mother, init, label="mixed init, device events", device=True)


def test_dynamic_without_lifecycle_equals_static_path(ctx):
    """No create or destroy: the dynamic pipeline and the static overlap check agree."""
    from paper_1910_11110_amd import vcheck as V
    lo, hi = gen.intervals(3000, 5, space=1 << 16, max_len=512)
    e = gen.plain_events(300_000, 3000, 6)
    st, fin, viol, nis = run_gpu(ctx, e, lo, hi, np.full(3000, O.NO_MOTHER, np.uint32))
    t = V.Trace.load(ctx, e, 3000)
    t.set_arrays(lo, hi)
    t.check()
    ctx.sync()
    assert np.array_equal(st, t.status()) and np.array_equal(fin, t.final())
    assert viol.total == t.violations().total and nis == t.induced_stuck()
    t.free()


@pytest.mark.parametrize("case", ["use-before-create", "use-after-destroy", "second-create", "destroy-dead",
                                  "mother-dead"])
def test_dynamic_lifetime_errors(ctx, case):
    """Lifetime errors are rejected with the oracle's index (host events: at set-up)."""
    from paper_1910_11110_amd import vcheck as V
    lo = np.array([0, 2, 4], np.uint32)
    hi = np.array([10, 5, 8], np.uint32)
    mo = np.array([O.NO_MOTHER, 0, 0], np.uint32)
    C, D = 6 << 24, 7 << 24
    traces = {
        "use-before-create": [0, 1, C | 1],
        "use-after-destroy": [C | 1, 1, D | 1, 0, 1],
        "second-create": [C | 1, D | 1, C | 1],
        "destroy-dead": [C | 1, D | 1, 2, D | 1],
        "mother-dead": [0, D | 0, C | 1],
    }
    ev = np.array(traces[case], np.uint32)
    with pytest.raises(O.OracleError) as want:
        O.check_dynamic(ev, lo, hi, mo)
    idx = str(want.value).split("index ")[1]
    t = V.Trace.load(ctx, ev, 3, lifetimes=True)
    with pytest.raises(V.VCError) as got:
        t.set_dynamic_arrays(lo, hi, mo)
    assert got.value.code == V.VC_EINVAL and f"index {idx}" in str(got.value)
    t.free()


def test_dynamic_layout_rejected(ctx):
    from paper_1910_11110_amd import vcheck as V
    lo = np.array([0, 2, 12], np.uint32)
    hi = np.array([10, 5, 14], np.uint32)
    t = V.Trace.load(ctx, np.zeros(4, np.uint32), 3, lifetimes=True)
    with pytest.raises(V.VCError) as e:
        t.set_dynamic_arrays(lo, hi, np.array([O.NO_MOTHER, 2, O.NO_MOTHER], np.uint32))
    assert e.value.code == V.VC_EINVAL and "array 1" in str(e.value)
    t.free()


def test_dynamic_rerun_is_deterministic(ctx):
    from paper_1910_11110_amd import vcheck as V
    d = gen.dynamic_trace(300_001, 16, 700, 9, space=1 << 15, max_len=1024)
    t = V.Trace.load(ctx, d.events, d.lo.size, lifetimes=True)
    t.set_dynamic_arrays(d.lo, d.hi, d.mother)
    outs = []
    for _ in range(3):
        t.check()
        ctx.sync()
        outs.append((t.status().copy(), t.final().copy(), t.violations().indices.copy()))
    t.free()
    for o in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(o, outs[0]))


@pytest.mark.timeout(600)
def test_dynamic_workload_full_size(ctx):
    """The measured workload: 2^24 events over 2^10 vectors and 64,512 partial vectors in
    a 2^24-element address space."""
    say("[dynamic] generating the full-size workload")
    d = gen.dynamic_trace(1 << 24, 1 << 10, (1 << 16) - (1 << 10), 0)
    sets = O.overlap_sets(d.lo, d.hi)
    assert_parity(ctx, d.events, d.lo, d.hi, d.mother, label="dynamic full size", sets=sets)


@pytest.mark.parametrize("n,nv,npv,space,maxlen", [(70_000, 4, 60, 1 << 12, 512), (600_000, 32, 2000, 1 << 16, 4096)])
def test_dynamic_bucket_and_sorted_routes_agree(ctx, n, nv, npv, space, maxlen):
    """The bucket-engine route (items as 32-bit words, two checks) and the sorted route
    (64-bit items, two scans) give the same bytes, from initial (I,I) statuses too."""
    import os
    d = gen.dynamic_trace(n, nv, npv, n + 3 * nv, space=space, max_len=maxlen)
    init = (np.arange(d.lo.size) % 4).astype(np.uint8)
    for ini in (None, init):
        a = run_gpu(ctx, d.events, d.lo, d.hi, d.mother, ini)
        os.environ["VC_GENERAL_PATH"] = "1"
        try:
            b = run_gpu(ctx, d.events, d.lo, d.hi, d.mother, ini)
        finally:
            del os.environ["VC_GENERAL_PATH"]
        assert np.array_equal(a[0], b[0]), "status bytes"
        assert np.array_equal(a[1], b[1]), "final statuses"
        assert a[2].total == b[2].total and np.array_equal(a[2].indices, b[2].indices), "violations"
        assert a[3] == b[3], "stuck induced"
