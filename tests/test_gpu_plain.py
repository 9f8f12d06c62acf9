"""Parity of the plain check (HIP path through the C ABI) with the oracle."""
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


def run_gpu(ctx, events, n_ids, init=None):
    from paper_1910_11110_amd import vcheck as V
    t = V.Trace.load(ctx, events, n_ids, init)
    t.check()
    ctx.sync()
    res = (t.status(), t.final(), t.violations())
    t.free()
    return res


def assert_parity(ctx, events, n_ids, init=None, label=""):
    say(f"[plain] {label} n={events.size} n_ids={n_ids}")
    st, fin, viol = run_gpu(ctx, events, n_ids, init)
    ref = O.check(events, n_ids, init)
    if not np.array_equal(st, ref.status):
        bad = np.nonzero(st != ref.status)[0]
        raise AssertionError(f"{label}: {bad.size} status bytes differ, first at {bad[0]}: "
                             f"gpu {st[bad[0]]:#x} oracle {ref.status[bad[0]]:#x}")
    assert np.array_equal(fin, ref.final), f"{label}: final status differs"
    assert viol.total == ref.violations.size and np.array_equal(viol.indices, ref.violations), label
    assert viol.first == ref.first, label


@pytest.mark.parametrize("seed", range(5))
def test_plain_small_workload(ctx, seed):
    """The 10,000-event, 64-variable plain workload, five seeds."""
    e = gen.plain_events(10_000, 64, seed)
    assert_parity(ctx, e, 64, label=f"plain-10k seed {seed}")


@pytest.mark.parametrize("n,n_ids", [(1, 1), (2, 1), (4095, 3), (4096, 64), (4097, 64), (65537, 1),
                                     (300_001, 7), (1 << 20, 64), (1_000_003, 1 << 16), (777_777, 1 << 21),
                                     (2_000_000, (1 << 24))])
def test_plain_shapes(ctx, n, n_ids):
    """Ragged tails, a single id, several tiles, and id spaces from 1 to 2^24."""
    e = gen.plain_events(n, n_ids, 100 + n % 97)
    assert_parity(ctx, e, n_ids, label=f"shape {n}x{n_ids}")


def test_plain_empty(ctx):
    from paper_1910_11110_amd import vcheck as V
    say("[plain] empty")
    t = V.Trace.load(ctx, np.zeros(0, np.uint32), 5)
    t.check()
    ctx.sync()
    assert t.status().size == 0
    assert list(t.final()) == [1] * 5
    v = t.violations()
    assert v.total == 0 and v.first == 0


def test_plain_initial_statuses(ctx):
    """Arbitrary initial statuses, including (I,I)."""
    n_ids = 1000
    init = gen.below(gen.draws(5, 77, 0, n_ids), 4).astype(np.uint8)
    e = gen.plain_events(200_000, n_ids, 5)
    assert_parity(ctx, e, n_ids, init=init, label="init-any")


def test_plain_device_input(ctx):
    """Events and init already in device memory (borrowed torch tensors)."""
    import torch
    e = gen.plain_events(500_000, 256, 9)
    init = gen.below(gen.draws(9, 78, 0, 256), 4).astype(np.uint8)
    from paper_1910_11110_amd import vcheck as V
    te = torch.from_numpy(e.view(np.int32)).cuda()
    ti = torch.from_numpy(init).cuda()
    torch.cuda.synchronize()
    say("[plain] device input")
    t = V.Trace.load(ctx, te, 256, ti)
    t.check()
    ctx.sync()
    ref = O.check(e, 256, init)
    assert np.array_equal(t.status(), ref.status)
    assert np.array_equal(t.final(), ref.final)
    t.free()


def test_plain_repeat_deterministic(ctx):
    """The same trace checked three times gives identical bytes (races would not)."""
    from paper_1910_11110_amd import vcheck as V
    e = gen.plain_events(3_000_000, 4096, 21)
    t = V.Trace.load(ctx, e, 4096)
    outs = []
    for _ in range(3):
        t.check()
        ctx.sync()
        outs.append(t.status().copy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    ref = O.check(e, 4096)
    assert np.array_equal(outs[0], ref.status)
    t.free()


def test_plain_invalid_device_event_reported(ctx):
    """A malformed event word in device memory is reported by vc_sync with its index."""
    import torch
    from paper_1910_11110_amd import vcheck as V
    e = gen.plain_events(10_000, 64, 1)
    e[1234] = (e[1234] & 0xFFFFFF) | (6 << 24)  # op 6 does not exist
    te = torch.from_numpy(e.view(np.int32)).cuda()
    torch.cuda.synchronize()
    t = V.Trace.load(ctx, te, 64)
    t.check()
    with pytest.raises(V.VCError) as ex:
        ctx.sync()
    assert "1234" in str(ex.value)
    t.free()


def test_plain_invalid_host_event_rejected(ctx):
    from paper_1910_11110_amd import vcheck as V
    e = gen.plain_events(100, 64, 1)
    e[7] = 70  # id 70 >= n_ids
    with pytest.raises(V.VCError) as ex:
        V.Trace.load(ctx, e, 64)
    assert ex.value.code == V.VC_EINVAL and "index 7" in str(ex.value)


@pytest.mark.parametrize("n,n_ids", [(10_000, 64), (4096 * 37 + 5, 64), (1 << 20, 17), (333_333, 1), (1 << 22, 64)])
def test_small_and_general_paths_agree(ctx, n, n_ids):
    """Traces over at most 64 ids take the single-kernel path; the general sort-based path
    (forced by VC_GENERAL_PATH) must give the same bytes, and both the oracle's."""
    import os
    e = gen.plain_events(n, n_ids, 300 + n_ids)
    init = gen.below(gen.draws(n, 79, 0, n_ids), 4).astype(np.uint8)
    assert_parity(ctx, e, n_ids, init=init, label=f"small path {n}x{n_ids}")
    os.environ["VC_GENERAL_PATH"] = "1"
    try:
        assert_parity(ctx, e, n_ids, init=init, label=f"general path {n}x{n_ids}")
    finally:
        del os.environ["VC_GENERAL_PATH"]


def test_small_path_misaligned_device_events(ctx):
    """A device buffer that is not 16-byte aligned takes the general path."""
    import torch
    from paper_1910_11110_amd import vcheck as V
    e = gen.plain_events(100_001, 64, 31)
    te = torch.from_numpy(np.concatenate([np.zeros(1, np.uint32), e]).view(np.int32)).cuda()[1:]
    torch.cuda.synchronize()
    t = V.Trace.load(ctx, te, 64)
    t.check()
    ctx.sync()
    ref = O.check(e, 64)
    assert np.array_equal(t.status(), ref.status)
    t.free()


@pytest.mark.parametrize("n,n_ids", [(4097, 65), (100_000, 4096), (100_000, 4097), (1 << 20, 12_345),
                                     (2_000_003, 1 << 20), (3_000_000, (1 << 22) - 3), (50_000, 1 << 22)])
def test_bucket_and_general_paths_agree(ctx, n, n_ids):
    """Id spaces above 64 take the bucket path (partition by id >> 12, per-bucket scan,
    replay); the general sort-based path must give the same bytes, and both the oracle's."""
    import os
    e = gen.plain_events(n, n_ids, 500 + n_ids % 101)
    init = gen.below(gen.draws(n, 80, 0, n_ids), 4).astype(np.uint8)
    assert_parity(ctx, e, n_ids, init=init, label=f"bucket path {n}x{n_ids}")
    os.environ["VC_GENERAL_PATH"] = "1"
    try:
        assert_parity(ctx, e, n_ids, init=init, label=f"general path {n}x{n_ids}")
    finally:
        del os.environ["VC_GENERAL_PATH"]


def test_bucket_path_skewed_ids(ctx):
    """Most events on a few ids of one bucket, the rest spread thin (long chains of
    tiles inside one bucket, many nearly empty buckets)."""
    n, n_ids = 3_000_000, 1 << 20
    e = gen.plain_events(n, n_ids, 77)
    hot = gen.plain_events(n, 50, 78)
    pick = gen.below(gen.draws(77, 81, 0, n), 10) < 8
    e = np.where(pick, hot, e).astype(np.uint32)
    assert_parity(ctx, e, n_ids, label="skewed")


def test_trace_outlives_context():
    """A trace whose context was destroyed can only be freed: other calls report
    VC_ESTATE, and freeing it later is safe."""
    from paper_1910_11110_amd import vcheck as V
    c = V.Context(0)
    t = V.Trace.load(c, gen.plain_events(5000, 64, 3), 64)
    t.check()
    c.close()
    with pytest.raises(V.VCError) as ex:
        t.info()
    assert ex.value.code == V.VC_ESTATE
    with pytest.raises(V.VCError):
        t.check()
    t.free()


@pytest.mark.timeout(600)
def test_small_path_full_size_persistent(ctx):
    """The plain law at 2^28 events over 64 ids (the single-trace measurement workload):
    32,768 tiles of 8,192 events, far more than the resident grid, so every workgroup of
    the <= 64-id kernel takes many tiles in turn."""
    say("[plain] generating 2^28 events over 64 ids")
    e = gen.plain_events(1 << 28, 64, 0)
    assert_parity(ctx, e, 64, label="plain 2^28 x 64")


@pytest.mark.timeout(600)
def test_bucket_path_full_size(ctx):
    """The plain law at 2^26 events over 2^20 ids (bucket path at its measured size)."""
    say("[plain] generating 2^26 events over 2^20 ids")
    e = gen.plain_events(1 << 26, 1 << 20, 0)
    assert_parity(ctx, e, 1 << 20, label="plain 2^26 x 2^20")
