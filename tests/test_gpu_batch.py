"""Batched check: many independent traces in one pipeline, each identical to the oracle and
to its own single-trace check."""
import os
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


def make_traces(n, seed, len_range=(100, 50_000), vars_range=(8, 65536), with_init=True):
    shapes = gen.trace_shapes(n, seed, len_range=len_range, vars_range=vars_range)
    out = []
    for i, sh in enumerate(shapes):
        ev, lo, hi = gen.trace_inputs(sh)
        init = None
        if with_init and i % 5 == 1:
            init = gen.below(gen.draws(sh.seed, 400, 0, sh.n_vars), 4).astype(np.uint8)
        out.append((ev, sh.n_vars, lo, hi, init))
    return out


def load_all(ctx, inputs):
    from paper_1910_11110_amd import vcheck as V
    traces = []
    for ev, nv, lo, hi, init in inputs:
        t = V.Trace.load(ctx, ev, nv, init)
        if lo is not None:
            t.set_arrays(lo, hi)
        traces.append(t)
    return traces


def oracle_of(ev, nv, lo, hi, init):
    if lo is None:
        return O.check(ev, nv, init)
    return O.check_overlap(ev, lo, hi, init)


def assert_trace(t, ref, label):
    st = t.status()
    if not np.array_equal(st, ref.status):
        bad = np.nonzero(st != ref.status)[0]
        raise AssertionError(f"{label}: {bad.size} statuses differ, first {bad[0]}")
    assert np.array_equal(t.final(), ref.final), f"{label}: final"
    v = t.violations()
    assert v.total == ref.violations.size and np.array_equal(v.indices, ref.violations), f"{label}: violations"
    assert v.first == ref.first, label
    assert t.induced_stuck() == ref.n_induced_stuck, label


def test_batch_small_mixed(ctx):
    from paper_1910_11110_amd import vcheck as V
    inputs = make_traces(40, 1)
    traces = load_all(ctx, inputs)
    say("[batch] 40 mixed traces")
    V.batch_check(ctx, traces)
    ctx.sync()
    for i, (t, inp) in enumerate(zip(traces, inputs)):
        assert_trace(t, oracle_of(*inp), f"trace {i}")
    # replay of the captured graph gives identical bytes
    first = [t.status().copy() for t in traces]
    V.batch_check(ctx, traces)
    ctx.sync()
    assert all(np.array_equal(a, t.status()) for a, t in zip(first, traces))
    g = C_info(V, ctx)
    say(f"[batch] graph={g}")
    for t in traces:
        t.free()


def C_info(V, ctx):
    import ctypes as C
    g, b, gc, sg = C.c_int(), C.c_int(), C.c_uint(), C.c_uint()
    V._check(V.lib().vc_batch_info(ctx.h, C.byref(g), C.byref(b), C.byref(gc), C.byref(sg)))
    return g.value, b.value, gc.value, sg.value


def test_batch_equals_alone(ctx):
    """A trace checked alone and inside a batch gives the same bytes."""
    from paper_1910_11110_amd import vcheck as V
    inputs = make_traces(12, 2)
    traces = load_all(ctx, inputs)
    V.batch_check(ctx, traces)
    ctx.sync()
    in_batch = [(t.status().copy(), t.final().copy()) for t in traces]
    for t, (s, f) in zip(traces, in_batch):
        t.check()
        ctx.sync()
        assert np.array_equal(t.status(), s) and np.array_equal(t.final(), f)
        t.free()


def test_batch_edge_cases(ctx):
    """Empty traces, one-event traces, a single id, and a batch of one."""
    from paper_1910_11110_amd import vcheck as V
    inputs = [(np.zeros(0, np.uint32), 3, None, None, None),
              (gen.plain_events(1, 1, 3), 1, None, None, None),
              (gen.plain_events(4097, 1, 4), 1, None, None, None),
              (np.zeros(0, np.uint32), 1, None, None, None),
              (gen.plain_events(5000, 70, 5), 70, None, None, np.zeros(70, np.uint8))]
    traces = load_all(ctx, inputs)
    V.batch_check(ctx, traces)
    ctx.sync()
    for i, (t, inp) in enumerate(zip(traces, inputs)):
        assert_trace(t, oracle_of(*inp), f"edge {i}")
    V.batch_check(ctx, traces[4:])
    ctx.sync()
    assert_trace(traces[4], oracle_of(*inputs[4]), "batch of one")
    for t in traces:
        t.free()


def test_batch_autotuner_is_parity_clean(ctx, tmp_path):
    """With tuning on, every candidate setting of the sorted route (the one with a sort to
    tune) runs on the batch; the chosen one gives the oracle's bytes and is cached per
    shape."""
    from paper_1910_11110_amd import vcheck as V
    cache = tmp_path / "tune.json"
    os.environ["VC_AUTOTUNE"] = "1"
    os.environ["VC_TUNE_CACHE"] = str(cache)
    os.environ["VC_GENERAL_PATH"] = "1"
    try:
        inputs = make_traces(25, 3)
        traces = load_all(ctx, inputs)
        V.batch_check(ctx, traces)
        ctx.sync()
        for i, (t, inp) in enumerate(zip(traces, inputs)):
            assert_trace(t, oracle_of(*inp), f"tuned trace {i}")
        assert cache.exists() and "gfx950" in cache.read_text()
        say(f"[batch] tuned: {C_info(V, ctx)} cache {cache.read_text().strip()}")
        for t in traces:
            t.free()
    finally:
        del os.environ["VC_AUTOTUNE"]
        del os.environ["VC_TUNE_CACHE"]
        del os.environ["VC_GENERAL_PATH"]


# array traces are compared with the oracle while the oracle's O(n^2) overlap-set
# construction over them stays within this many pair tests (about 20 s on 16 host
# threads); the traces with the most arrays beyond it are compared with their own
# single-trace check instead
ORACLE_PAIR_BUDGET = 5e10


def _oracle_many(jobs):
    """Oracle results of (events, n_ids, lo, hi, init) jobs, on a pool of host threads
    (the oracle runs in C and releases the interpreter lock)."""
    import concurrent.futures as cf
    workers = min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda j: oracle_of(*j), jobs))


@pytest.mark.timeout(900)
def test_batch_workload_full_size(ctx):
    """The batched workload at full size: 4,096 traces, lengths log-uniform in [100, 10^6],
    variables log-uniform in [8, 65,536], 20 % with intervals.  Every trace without arrays
    and every array trace within the oracle's pair budget is compared with the oracle in
    full (statuses, final table, violations); the remaining array traces (the ones with the
    most arrays) are compared with their own single-trace check."""
    from paper_1910_11110_amd import vcheck as V
    say("[batch] generating 4096 traces")
    shapes = gen.trace_shapes(4096, 0)
    traces, inputs = [], []
    for sh in shapes:
        ev, lo, hi = gen.trace_inputs(sh)
        t = V.Trace.load(ctx, ev, sh.n_vars)
        if lo is not None:
            t.set_arrays(lo, hi)
        traces.append(t)
        inputs.append((ev, sh.n_vars, lo, hi, None))
    say(f"[batch] {sum(s.length for s in shapes)} events; running")
    V.batch_check(ctx, traces)
    ctx.sync()
    arr = sorted((i for i, sh in enumerate(shapes) if sh.has_arrays), key=lambda i: shapes[i].n_vars)
    pairs, in_budget = 0.0, set()
    for i in arr:
        pairs += float(shapes[i].n_vars) ** 2
        if pairs > ORACLE_PAIR_BUDGET:
            break
        in_budget.add(i)
    cmp = [i for i, sh in enumerate(shapes) if not sh.has_arrays or i in in_budget]
    rest = [i for i in arr if i not in in_budget]
    say(f"[batch] oracle on {len(cmp)} traces ({len(in_budget)} of {len(arr)} with arrays); "
        f"{len(rest)} array traces against their single-trace check")
    for a in range(0, len(cmp), 512):
        part = cmp[a:a + 512]
        refs = _oracle_many([inputs[i] for i in part])
        for i, ref in zip(part, refs):
            assert_trace(traces[i], ref, f"full trace {i}")
        say(f"[batch] {a + len(part)} traces match the oracle")
    batched = {i: (traces[i].status().copy(), traces[i].final().copy(), traces[i].violations()) for i in rest}
    for i in rest:
        traces[i].check()
        ctx.sync()
        s0, f0, v0 = batched[i]
        assert np.array_equal(traces[i].status(), s0) and np.array_equal(traces[i].final(), f0), f"alone {i}"
        v1 = traces[i].violations()
        assert v1.total == v0.total and np.array_equal(v1.indices, v0.indices) and v1.first == v0.first
    for t in traces:
        t.free()


def _route_results(ctx, inputs, general):
    from paper_1910_11110_amd import vcheck as V
    if general:
        os.environ["VC_GENERAL_PATH"] = "1"
    try:
        traces = load_all(ctx, inputs)
        V.batch_check(ctx, traces)
        ctx.sync()
        out = [(t.status().copy(), t.final().copy(), t.violations().indices.copy(), t.induced_stuck()) for t in traces]
    finally:
        os.environ.pop("VC_GENERAL_PATH", None)
    for t in traces:
        t.free()
    return out


def test_batch_bucket_and_sorted_routes_agree(ctx):
    """The bucket-engine route (groups of traces as 32-bit words) and the sorted route give
    the same bytes on a mixed batch with arrays and initial statuses."""
    inputs = make_traces(30, 7)
    say("[batch] 30 traces through both routes")
    a = _route_results(ctx, inputs, False)
    b = _route_results(ctx, inputs, True)
    for i, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x[0], y[0]), f"trace {i}: statuses"
        assert np.array_equal(x[1], y[1]), f"trace {i}: final"
        assert np.array_equal(x[2], y[2]), f"trace {i}: violations"
        assert x[3] == y[3], f"trace {i}: induced stuck"


def test_batch_groups_split_at_the_key_space(ctx):
    """Traces whose ids together exceed one bucket engine's key space (2^22) are checked in
    several groups; every trace equals the oracle, the one with arrays included."""
    from paper_1910_11110_amd import vcheck as V
    big = 3 << 19  # three of these exceed 2^22 together
    inputs = [(gen.plain_events(200_000, big, 11 + k), big, None, None,
               gen.below(gen.draws(11 + k, 400, 0, big), 4).astype(np.uint8) if k == 1 else None) for k in range(3)]
    n_arr = 300
    lo, hi = gen.intervals(n_arr, 21)
    inputs.insert(2, (gen.plain_events(50_000, n_arr, 22), n_arr, lo, hi, None))
    traces = load_all(ctx, inputs)
    say("[batch] 4 traces over more than 2^22 ids")
    V.batch_check(ctx, traces)
    ctx.sync()
    for i, (t, inp) in enumerate(zip(traces, inputs)):
        assert_trace(t, oracle_of(*inp), f"trace {i}")
    for t in traces:
        t.free()


def test_batch_malformed_device_event_reported_alone(ctx):
    """A malformed event word in one trace's device memory is reported for that trace
    (with its index) by the sync after a batched check; the other traces of the batch,
    one with arrays, still equal the oracle."""
    import torch
    from paper_1910_11110_amd import vcheck as V
    inputs = make_traces(6, 9, len_range=(5000, 40000), with_init=False)
    ev, nv, lo, hi, init = inputs[2]
    bad = ev.copy()
    bad[77] = (bad[77] & 0xFFFFFF) | (6 << 24)  # op 6 does not exist
    tb = torch.from_numpy(bad.view(np.int32)).cuda()
    torch.cuda.synchronize()
    traces = load_all(ctx, inputs[:2]) + [V.Trace.load(ctx, tb, nv)] + load_all(ctx, inputs[3:])
    if lo is not None:
        traces[2].set_arrays(lo, hi)
    say("[batch] 6 traces, one with a malformed device event")
    V.batch_check(ctx, traces)
    with pytest.raises(V.VCError) as ex:
        ctx.sync()
    assert "77" in str(ex.value)
    for i, (t, inp) in enumerate(zip(traces, inputs)):
        if i != 2:
            assert_trace(t, oracle_of(*inp), f"trace {i}")
    for t in traces:
        t.free()


def test_batch_dense_overlaps(ctx):
    """A batch with a trace whose arrays nearly all overlap (hundreds of induced items per
    write, spanning several steps of a chunk's 64-item walk) between plain traces: every
    trace equals the oracle, through the bucket route and the sorted route."""
    rng = np.random.default_rng(6)
    lo = rng.integers(0, 500, 300).astype(np.uint32)
    hi = (lo + rng.integers(300, 500, 300)).astype(np.uint32)
    inputs = make_traces(4, 10, len_range=(3000, 30000), with_init=False)
    inputs.insert(2, (gen.plain_events(9_000, 300, 15), 300, lo, hi, None))
    for general in (False, True):
        if general:
            os.environ["VC_GENERAL_PATH"] = "1"
        try:
            from paper_1910_11110_amd import vcheck as V
            traces = load_all(ctx, inputs)
            V.batch_check(ctx, traces)
            ctx.sync()
            for i, (t, inp) in enumerate(zip(traces, inputs)):
                assert_trace(t, oracle_of(*inp), f"trace {i} (general {general})")
            for t in traces:
                t.free()
        finally:
            os.environ.pop("VC_GENERAL_PATH", None)


def test_batch_bucket_route_autotuner(ctx, tmp_path):
    """The bucket route's settings (ids per group, events per chunk) are chosen by timing
    every candidate on the batch itself and cached per shape; the chosen one gives the
    oracle's bytes, and a second batch of the same shape takes the cached choice."""
    from paper_1910_11110_amd import vcheck as V
    cache = tmp_path / "tune.json"
    os.environ["VC_TUNE_CACHE"] = str(cache)
    try:
        inputs = make_traces(25, 4)
        traces = load_all(ctx, inputs)
        V.batch_check(ctx, traces)
        ctx.sync()
        for i, (t, inp) in enumerate(zip(traces, inputs)):
            assert_trace(t, oracle_of(*inp), f"tuned trace {i}")
        text = cache.read_text()
        assert "bucket:gfx950" in text, text
        say(f"[batch] bucket route tuned: {text.strip()}")
        # the batch info gives the bucket route's settings: ids per group (a power of two)
        # and events per chunk of a trace without arrays, among the candidates
        graph, bits, chunk, scan = C_info(V, ctx)
        assert bits in (20, 21, 22) and chunk in (4096, 16384) and scan == 0, (bits, chunk, scan)
        for t in traces:
            t.free()
        traces = load_all(ctx, inputs)  # same shape, new handles: the cached choice
        V.batch_check(ctx, traces)
        ctx.sync()
        for i, (t, inp) in enumerate(zip(traces, inputs)):
            assert_trace(t, oracle_of(*inp), f"cached trace {i}")
        for t in traces:
            t.free()
    finally:
        del os.environ["VC_TUNE_CACHE"]
