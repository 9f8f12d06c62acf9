"""Parity of the well-declaredness check (HIP path through the C ABI) with the oracle:
every component's verdict byte and the list of components that are not well-declared."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen
from tests.helpers import load_yaml
from tests.test_oracle_declared import _case

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


def run_gpu(ctx, co, de, nv, bo, bd, idx=None, lo=None, hi=None, extend=False, device=False):
    from paper_1910_11110_amd import vcheck as V
    if device:
        import torch
        co, de, bo, bd = (torch.from_numpy(np.ascontiguousarray(a).view(np.int64 if a.dtype == np.uint64 else np.int32))
                          .cuda() for a in (co, de, bo, bd))
        if idx is not None:
            idx = torch.from_numpy(idx.view(np.int32)).cuda()
    t = V.check_declared(ctx, co, de, nv, bo, bd, idx, lo, hi, extend)
    ctx.sync()
    res = (t.status(), t.violations())
    t.free()
    return res


def assert_parity(ctx, p, extend=False, label="", device=False):
    say(f"[declared] {label}: {p.comp_off.size - 1} components, {p.body.size} body events, extend={extend}")
    v, ill = run_gpu(ctx, p.comp_off, p.decls, p.n_vars, p.body_off, p.body, p.idx, p.lo, p.hi, extend, device)
    sets = O.overlap_sets(p.lo, p.hi) if p.lo is not None and p.lo.size > 4096 else None
    ref = O.check_declared(p.comp_off, p.decls, p.n_vars, p.body_off, p.body, p.idx, p.lo, p.hi, extend, sets)
    if not np.array_equal(v, ref):
        i = int(np.nonzero(v != ref)[0][0])
        raise AssertionError(f"{label}: verdicts differ first at component {i}: gpu {v[i]:#x} oracle {ref[i]:#x}")
    want = np.nonzero(ref)[0]
    assert ill.total == want.size and np.array_equal(ill.indices, want), label
    assert ill.first == (int(want[0]) if want.size else ref.size), label


@pytest.mark.parametrize("ex", load_yaml("declared_examples.yaml"), ids=lambda e: e["name"])
def test_declared_examples(ctx, ex):
    co, de, nv, bo, bd, idx, lo, hi = _case(ex)
    v, _ = run_gpu(ctx, co, de, nv, bo, bd, idx, lo, hi)
    assert np.array_equal(v, O.check_declared(co, de, nv, bo, bd, idx, lo, hi)), ex["name"]


@pytest.mark.parametrize("n_comp,n_vars,arrays,extend", [(1, 1, False, False), (257, 8, False, False),
                                                         (40_003, 1000, False, False), (300_001, 1 << 20, False, False),
                                                         (3, 4, True, False), (20_001, 2000, True, False),
                                                         (20_001, 2000, True, True), (200_003, 1 << 16, True, True)])
def test_declared_shapes(ctx, n_comp, n_vars, arrays, extend):
    space = max(64, n_vars * 8) if arrays else 1 << 24
    p = gen.declared_program(n_comp, n_vars, n_comp + n_vars, arrays=arrays, space=space, max_len=32,
                             kmax=min(4, n_vars), p_err=0.1)
    assert_parity(ctx, p, extend, label=f"{n_comp} components")


def test_declared_empty_components_and_bodies(ctx):
    co = np.array([0, 0, 2, 2, 3], np.uint64)
    de = np.array([1, 2 | (1 << 24), 0 | (2 << 24) | (1 << 27)], np.uint32)
    bo = np.array([0, 1, 1, 3, 3], np.uint64)
    bd = np.array([0, 1, 2 | (1 << 24)], np.uint32)
    from oracle.oracle import check_declared
    v, ill = run_gpu(ctx, co, de, 3, bo, bd)
    assert np.array_equal(v, check_declared(co, de, 3, bo, bd))


def test_declared_device_input(ctx):
    p = gen.declared_program(50_000, 3000, 4, arrays=True, space=1 << 15, max_len=32, p_err=0.1)
    assert_parity(ctx, p, True, label="device input", device=True)


@pytest.mark.parametrize("case", ["repeated-var", "bad-body-word", "index-out-of-range", "decl-before-body"])
def test_declared_malformed(ctx, case):
    from paper_1910_11110_amd import vcheck as V
    lo, hi = np.array([0, 4, 9], np.uint32), np.array([4, 8, 12], np.uint32)
    co = np.array([0, 1, 3], np.uint64)
    de = np.array([0, 1, 2 | (1 << 24)], np.uint32)
    bo = np.array([0, 1, 3], np.uint64)
    bd = np.array([0, 1, 2 | (1 << 24)], np.uint32)
    idx = np.array([0, 1, 2], np.uint32)
    if case == "repeated-var":
        de[2] = 1 | (1 << 24)
    elif case == "bad-body-word":
        bd[2] = 2 | (5 << 24)
    elif case == "index-out-of-range":
        idx[1] = 4
    else:  # a bad declaration in component 1 and a bad body word in component 0: the body word first
        de[2] = 1 | (1 << 24)
        idx[0] = 9
    with pytest.raises(O.OracleError) as want:
        O.check_declared(co, de, 3, bo, bd, idx, lo, hi)
    with pytest.raises(V.VCError) as got:
        V.check_declared(ctx, co, de, 3, bo, bd, idx, lo, hi)
    assert got.value.code == V.VC_EINVAL and str(want.value) in str(got.value)


@pytest.mark.timeout(600)
def test_declared_workload_full_size(ctx):
    """The measured workload: 2^20 components over 2^16 arrays, checked against O(M)."""
    say("[declared] generating the full-size workload")
    p = gen.declared_program(1 << 20, 1 << 16, 0, arrays=True, space=1 << 22, max_len=64)
    assert_parity(ctx, p, True, label="full size")


@pytest.mark.parametrize("kmax", [12, 16, 24])
def test_declared_wide_components(ctx, kmax):
    """Components with many declarations: a tile of 64 components then has fewer than the
    512 declarations the body walk stages in LDS (kmax 12), more (kmax 24), or either
    (kmax 16), so both the staged and the global reading of the declarations run;
    scalars, arrays, and arrays with the extension."""
    for arrays, extend in ((False, False), (True, False), (True, True)):
        p = gen.declared_program(6_001, 2000, 7 + kmax, arrays=arrays, space=1 << 14, max_len=32, kmax=kmax,
                                 p_err=0.1)
        assert_parity(ctx, p, extend, label=f"kmax {kmax} arrays {arrays} extend {extend}")
