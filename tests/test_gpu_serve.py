"""Serving: streams of chunks with resident status tables and continuous batching.
Each stream's results equal the oracle on the stream's whole trace, alone and in a mix."""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen

pytestmark = pytest.mark.gpu

CHUNK = 1 << 12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1910_11110_amd import vcheck as V
    c = V.Context(0)
    yield c
    c.close()


def run_streams(srv, specs, timeout=120.0, chunk=None):
    """specs: list of (events, n_ids, lo, hi, init).  Submits every chunk of every stream,
    interleaved, and returns per stream (status bytes, completions, final table)."""
    CHUNK = chunk or globals()["CHUNK"]
    sids, bufs, comps = [], [], {}
    for ev, n_ids, lo, hi, init in specs:
        sids.append(srv.open(n_ids, lo, hi, init))
        bufs.append(np.zeros(ev.size, np.uint8))
    chunk_of = {}
    maxc = max((ev.size + CHUNK - 1) // CHUNK for ev, *_ in specs)
    for k in range(maxc):
        for i, (ev, *_r) in enumerate(specs):
            a = k * CHUNK
            if a < ev.size:
                b = min(ev.size, a + CHUNK)
                cid = srv.submit(sids[i], ev[a:b], bufs[i][a:b])
                chunk_of[cid] = (i, a, b)
    want = len(chunk_of)
    got = []
    t0 = time.time()
    while len(got) < want:
        got += srv.poll()
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.001)
    for c in got:
        assert c.status == 0, f"chunk {c.chunk} failed with {c.status}"
        comps.setdefault(chunk_of[c.chunk][0], []).append(c)
    finals = [srv.close_stream(s, specs[i][1]) for i, s in enumerate(sids)]
    return bufs, comps, finals, got


def oracle_of(ev, n_ids, lo, hi, init):
    return O.check(ev, n_ids, init) if lo is None else O.check_overlap(ev, lo, hi, init)


def mixed_specs(n, seed):
    shapes = gen.trace_shapes(n, seed, len_range=(100, 60_000), vars_range=(8, 65536))
    specs = []
    for i, sh in enumerate(shapes):
        ev, lo, hi = gen.trace_inputs(sh)
        init = gen.below(gen.draws(sh.seed, 401, 0, sh.n_vars), 4).astype(np.uint8) if i % 4 == 3 else None
        specs.append((ev, sh.n_vars, lo, hi, init))
    return specs


def test_served_streams_match_oracle(ctx):
    from paper_1910_11110_amd import vcheck as V
    srv = V.Server(ctx, 64 << 30)
    specs = mixed_specs(24, 5)
    say("[serve] 24 streams")
    bufs, comps, finals, _ = run_streams(srv, specs)
    for i, spec in enumerate(specs):
        ref = oracle_of(*spec)
        assert np.array_equal(bufs[i], ref.status), f"stream {i} status"
        assert np.array_equal(finals[i], ref.final), f"stream {i} final"
        nv = sum(c.n_violations for c in comps.get(i, []))
        assert nv == ref.violations.size, f"stream {i} violations"
        firsts = [c.first_violation for c in comps.get(i, []) if c.n_violations]
        if firsts:
            assert min(firsts) == ref.first
        for c in comps.get(i, []):
            assert c.t_submit <= c.t_start <= c.t_done
        # a stream's chunks complete in order (one of them in flight at a time)
        assert [c.first_event for c in comps.get(i, [])] == sorted(c.first_event for c in comps.get(i, []))
    srv.close()


def test_served_alone_equals_in_mix(ctx):
    """Each stream's bytes are the same when it is served alone and among many others."""
    from paper_1910_11110_amd import vcheck as V
    specs = mixed_specs(16, 6)
    srv = V.Server(ctx, 64 << 30)
    mix_bufs, _, mix_finals, got = run_streams(srv, specs)
    srv.close()
    # at least one launch carried chunks of several streams (continuous batching)
    starts = {}
    for c in got:
        starts.setdefault(c.t_start, set()).add(c.stream)
    assert max(len(v) for v in starts.values()) > 1
    for i, spec in enumerate(specs[:6]):
        srv = V.Server(ctx, 64 << 30)
        alone, _, fin, _ = run_streams(srv, [spec])
        srv.close()
        assert np.array_equal(alone[0], mix_bufs[i]) and np.array_equal(fin[0], mix_finals[i]), f"stream {i}"


def test_served_admission_under_small_budget(ctx):
    """A budget that holds only a few chunks at a time: chunks wait, nothing is lost, and
    a chunk that can never fit is refused at submission."""
    from paper_1910_11110_amd import vcheck as V
    specs = mixed_specs(8, 7)
    budget = 3 * (45 * CHUNK) + 8 * 65536 + 4096
    srv = V.Server(ctx, budget)
    bufs, comps, finals, _ = run_streams(srv, specs)
    for i, spec in enumerate(specs):
        ref = oracle_of(*spec)
        assert np.array_equal(bufs[i], ref.status) and np.array_equal(finals[i], ref.final)
    s = srv.open(8)
    with pytest.raises(V.VCError) as ex:
        srv.submit(s, gen.plain_events(1 << 20, 8, 1))
    assert ex.value.code == V.VC_EBUDGET
    srv.close_stream(s, 8)
    srv.close()


def test_served_malformed_chunk_rejected(ctx):
    from paper_1910_11110_amd import vcheck as V
    srv = V.Server(ctx, 1 << 30)
    s = srv.open(16)
    e = gen.plain_events(100, 16, 2)
    e[10] = 99  # id >= n_ids
    with pytest.raises(V.VCError) as ex:
        srv.submit(s, e)
    assert ex.value.code == V.VC_EINVAL and "index 10" in str(ex.value)
    srv.close_stream(s, 16)
    srv.close()


@pytest.mark.timeout(600)
def test_served_workload_shapes_full_chunks(ctx):
    """Streams with the batched workload's shapes (lengths log-uniform in [100, 10^6],
    variables log-uniform in [8, 65,536], 20 % with intervals) submitted in chunks of
    2^16 events: every stream equals the oracle on its whole trace, and streams served
    alone give the same bytes as in the mix."""
    from paper_1910_11110_amd import vcheck as V
    shapes = gen.trace_shapes(40, 11)
    specs = []
    for i, sh in enumerate(shapes):
        ev, lo, hi = gen.trace_inputs(sh)
        specs.append((ev, sh.n_vars, lo, hi, None))
    n = sum(sp[0].size for sp in specs)
    say(f"[serve] 40 streams, {n} events, 2^16-event chunks")
    srv = V.Server(ctx, 64 << 30)
    bufs, comps, finals, got = run_streams(srv, specs, timeout=300.0, chunk=1 << 16)
    srv.close()
    starts = {}
    for c in got:
        starts.setdefault(c.t_start, set()).add(c.stream)
    assert max(len(v) for v in starts.values()) > 1
    for i, spec in enumerate(specs):
        ref = oracle_of(*spec)
        assert np.array_equal(bufs[i], ref.status), f"stream {i} status"
        assert np.array_equal(finals[i], ref.final), f"stream {i} final"
        assert sum(c.n_violations for c in comps.get(i, [])) == ref.violations.size, f"stream {i} violations"
    longest = sorted(range(len(specs)), key=lambda i: -specs[i][0].size)[:4]
    for i in longest:
        srv = V.Server(ctx, 64 << 30)
        alone, _, fin, _ = run_streams(srv, [specs[i]], timeout=300.0, chunk=1 << 16)
        srv.close()
        assert np.array_equal(alone[0], bufs[i]) and np.array_equal(fin[0], finals[i]), f"alone {i}"


def test_served_batches_split_at_the_id_limit(ctx):
    """Seventeen streams of 2^24 ids each hold more ids together than one batched launch
    takes (2^28): admission splits them over several launches, and every chunk completes
    with the oracle's results."""
    from paper_1910_11110_amd import vcheck as V
    specs = [(gen.plain_events(3000, 1 << 24, 900 + i), 1 << 24, None, None, None) for i in range(17)]
    srv = V.Server(ctx, 64 << 30)
    bufs, comps, finals, got = run_streams(srv, specs, chunk=1000)
    srv.close()
    starts = {}
    for c in got:
        starts.setdefault(c.t_start, set()).add(c.stream)
    assert max(len(v) for v in starts.values()) <= 16
    for i, spec in enumerate(specs):
        ref = oracle_of(*spec)
        assert np.array_equal(bufs[i], ref.status) and np.array_equal(finals[i], ref.final), f"stream {i}"
