"""Parity of the check over k memory spaces (HIP path through the C ABI) with the
oracle: every uint16 status, the final codes and the violations."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen
from tests.test_oracle_spaces import as_spaces

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


def run_gpu(ctx, ev, n_ids, k, init=None):
    from paper_1910_11110_amd import vcheck as V
    t = V.Trace.load_spaces(ctx, ev, n_ids, k, init)
    t.check()
    ctx.sync()
    res = (t.status16(), t.final(), t.violations())
    t.free()
    return res


def assert_parity(ctx, ev, n_ids, k, init=None, label=""):
    say(f"[spaces] {label}: n={ev.size} n_ids={n_ids} k={k}")
    st, fin, viol = run_gpu(ctx, ev, n_ids, k, init)
    ref = O.check_spaces(ev, n_ids, k, init)
    if not np.array_equal(st, ref.status):
        i = int(np.nonzero(st != ref.status)[0][0])
        raise AssertionError(f"{label}: statuses differ first at {i}: gpu {st[i]:#x} oracle {ref.status[i]:#x}")
    assert np.array_equal(fin, ref.final), f"{label}: final codes differ"
    assert viol.total == ref.violations.size and np.array_equal(viol.indices, ref.violations), label
    assert viol.first == ref.first, label


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("n,n_ids", [(1, 1), (4095, 3), (4097, 64), (300_001, 1000), (2_000_003, 1 << 20),
                                     (777_777, 1 << 24)])
def test_spaces_shapes(ctx, k, n, n_ids):
    assert_parity(ctx, gen.space_events(n, n_ids, k, n + k), n_ids, k, label=f"k={k}")


@pytest.mark.parametrize("k", [2, 3, 4])
def test_spaces_initial_codes(ctx, k):
    e = gen.space_events(500_000, 300, k, 40 + k)
    init = (np.arange(300) % (1 << k)).astype(np.uint8)
    assert_parity(ctx, e, 300, k, init, label=f"init codes k={k}")


def test_two_spaces_equal_the_plain_path(ctx):
    """k = 2 on the plain law written as copies equals the plain check's statuses."""
    from paper_1910_11110_amd import vcheck as V
    e = gen.plain_events(400_000, 5000, 3)
    st, fin, viol = run_gpu(ctx, as_spaces(e), 5000, 2)
    t = V.Trace.load(ctx, e, 5000)
    t.check()
    ctx.sync()
    s2 = t.status()
    assert np.array_equal(st & 0xF, s2 & 3) and np.array_equal((st >> 4) & 0xF, (s2 >> 2) & 3)
    assert np.array_equal(st >> 15, s2 >> 7) and np.array_equal(fin, t.final())
    assert np.array_equal(viol.indices, t.violations().indices)
    t.free()


def test_spaces_malformed_words(ctx):
    from paper_1910_11110_amd import vcheck as V
    import torch
    e = gen.space_events(10_000, 16, 3, 5)
    e[7777] = (e[7777] & np.uint32(0x00FFFFFF)) | np.uint32((2 << 24) | (3 << 28))  # copy to location 3 of 3
    with pytest.raises(V.VCError) as ex:
        V.Trace.load_spaces(ctx, e, 16, 3)
    assert ex.value.code == V.VC_EINVAL and "index 7777" in str(ex.value)
    t = V.Trace.load_spaces(ctx, torch.from_numpy(e.view(np.int32)).cuda(), 16, 3)
    t.check()
    with pytest.raises(V.VCError) as ex:
        ctx.sync()
    assert ex.value.code == V.VC_EINVAL and "index 7777" in str(ex.value)
    t.free()
    with pytest.raises(V.VCError):
        V.Trace.load_spaces(ctx, e[:10], 16, 5)


@pytest.mark.timeout(600)
def test_spaces_workload_full_size(ctx):
    """The measured workload: 2^26 events over 2^20 variables, k = 4."""
    say("[spaces] generating 2^26 events")
    assert_parity(ctx, gen.space_events(1 << 26, 1 << 20, 4, 0), 1 << 20, 4, label="spaces full size")
