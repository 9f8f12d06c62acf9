"""The allocation-free plain check (vc_check_small_noalloc) against the existing entry
point (vc_trace_load + vc_check) on the same inputs: status bytes, final statuses,
violation indices, count and first index, bit for bit.  Two calls in a row share the
library's one work space; the second has a smaller input, so anything the first call
left there must not leak into it."""
import sys

import numpy as np
import pytest

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


def existing(ctx, events, n_ids, init):
    from paper_1910_11110_amd import vcheck as V
    t = V.Trace.load(ctx, events, n_ids, init)
    t.check()
    ctx.sync()
    res = (t.status(), t.final(), t.violations())
    t.free()
    return res


def no_alloc(ctx, events, n_ids, init):
    import torch

    from paper_1910_11110_amd import vcheck as V
    dev = torch.device("cuda", 0)
    n = events.size
    ev = torch.from_numpy(events.view(np.int32)).to(dev)
    ini = None if init is None else torch.from_numpy(init).to(dev)
    # outputs pre-filled with garbage: every byte the call reports must be written by it
    status = torch.full((max(n, 1),), 0x5A, dtype=torch.uint8, device=dev)
    final = torch.full((n_ids,), 0x5A, dtype=torch.uint8, device=dev)
    viol = torch.full((max(n, 1),), -1, dtype=torch.int32, device=dev)
    counts = torch.full((3,), -7, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    V.check_small_noalloc(ctx, ev, n_ids, ini, status[:n], final, viol, counts)
    ctx.sync()
    c = counts.cpu().numpy().view(np.uint64)
    nv = int(c[0])
    return (status[:n].cpu().numpy(), final.cpu().numpy(), viol[:nv].cpu().numpy().view(np.uint32), nv, int(c[1]),
            int(c[2]))


def compare(ctx, events, n_ids, init, label):
    say(f"[no-alloc] {label}: n={events.size} n_ids={n_ids}")
    st0, fin0, v0 = existing(ctx, events, n_ids, init)
    st1, fin1, v1, nv, first, bad = no_alloc(ctx, events, n_ids, init)
    assert bad == (1 << 64) - 1, f"{label}: malformed index {bad} reported"
    if not np.array_equal(st0, st1):
        i = int(np.nonzero(st0 != st1)[0][0])
        raise AssertionError(f"{label}: status bytes differ first at {i}: {st0[i]:#x} vs {st1[i]:#x}")
    assert np.array_equal(fin0, fin1), f"{label}: final statuses differ"
    assert nv == v0.total and np.array_equal(v1, v0.indices), f"{label}: violations differ"
    assert first == v0.first, f"{label}: first violation {first} vs {v0.first}"


def test_no_alloc_matches_check_two_calls():
    """A large call (many tiles per workgroup, violations) then a smaller one with other
    initial statuses: both equal the existing entry point."""
    from paper_1910_11110_amd import vcheck as V
    ctx = V.Context(0)
    try:
        e1 = gen.plain_events(3_000_017, 64, 21)
        compare(ctx, e1, 64, None, "first call, 3,000,017 events over 64 ids")
        e2 = gen.plain_events(70_001, 37, 22)
        init = (np.arange(37) % 4).astype(np.uint8)
        compare(ctx, e2, 37, init, "second call, 70,001 events over 37 ids, mixed initial statuses")
    finally:
        ctx.close()


def test_no_alloc_limits_and_edges(ctx):
    """Sizes beyond the limits are rejected before anything runs; the largest accepted
    size, an empty trace and a one-event trace equal the existing entry point."""
    import torch

    from paper_1910_11110_amd import vcheck as V
    dev = torch.device("cuda", 0)
    z8 = torch.zeros(4, dtype=torch.uint8, device=dev)
    z32 = torch.zeros(4, dtype=torch.int32, device=dev)
    c3 = torch.zeros(3, dtype=torch.int64, device=dev)
    with pytest.raises(V.VCError) as ex:
        V.check_small_noalloc(ctx, z32, 65, None, z8, torch.zeros(65, dtype=torch.uint8, device=dev), z32, c3)
    assert ex.value.code == V.VC_EINVAL
    big = torch.zeros((1 << 24) + 4, dtype=torch.int32, device=dev)
    with pytest.raises(V.VCError) as ex:
        V.check_small_noalloc(ctx, big[: (1 << 24) + 1], 8, None, z8, z8, z32, c3)
    assert ex.value.code == V.VC_EINVAL and "exceeds" in str(ex.value)
    with pytest.raises(V.VCError) as ex:
        V.check_small_noalloc(ctx, big[1:9], 8, None, z8, z8, z32, c3)
    assert ex.value.code == V.VC_EINVAL and "aligned" in str(ex.value)
    del big
    compare(ctx, gen.plain_events(1 << 24, 64, 23), 64, None, "largest accepted size 2^24")
    compare(ctx, np.zeros(0, np.uint32), 5, None, "empty trace")
    compare(ctx, gen.plain_events(1, 1, 24), 1, None, "one event")


def test_no_alloc_reports_malformed_event(ctx):
    """A malformed device word (op 6) is reported through the counters, not by a fault."""
    import torch

    from paper_1910_11110_amd import vcheck as V
    dev = torch.device("cuda", 0)
    e = gen.plain_events(50_000, 16, 25)
    e[31_337] = (e[31_337] & np.uint32(0x08FFFFFF)) | np.uint32(6 << 24)
    ev = torch.from_numpy(e.view(np.int32)).to(dev)
    st = torch.empty(e.size, dtype=torch.uint8, device=dev)
    fin = torch.empty(16, dtype=torch.uint8, device=dev)
    viol = torch.empty(e.size, dtype=torch.int32, device=dev)
    counts = torch.zeros(3, dtype=torch.int64, device=dev)
    V.check_small_noalloc(ctx, ev, 16, None, st, fin, viol, counts)
    ctx.sync()
    assert int(counts.cpu().numpy().view(np.uint64)[2]) == 31_337
