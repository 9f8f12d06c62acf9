"""Parity of the translation of access-mode declarations (HIP path) with the oracle."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_11110_amd import gen
from tests.helpers import decl, ev, load_yaml, parse_events
from tests.test_oracle_pins import _components

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


def gpu_translate(ctx, comp_off, decls, n_vars, body_off=None, body=None, check=True):
    from paper_1910_11110_amd import vcheck as V
    t = V.translate(ctx, comp_off, decls, n_vars, body_off, body, check=check)
    ctx.sync()
    return t


def assert_translation(ctx, comp_off, decls, n_vars, body_off=None, body=None, label=""):
    say(f"[translate] {label} comps={len(comp_off) - 1} decls={len(decls)} n_vars={n_vars}")
    t = gpu_translate(ctx, comp_off, decls, n_vars, body_off, body)
    ref_tr = O.translate(comp_off, decls, n_vars, body_off, body)
    got = t.events()
    assert got.size == ref_tr.size, f"{label}: {got.size} vs {ref_tr.size} events"
    if not np.array_equal(got, ref_tr):
        bad = np.nonzero(got != ref_tr)[0]
        raise AssertionError(f"{label}: translated trace differs at {bad.size} events, first {bad[0]}: "
                             f"gpu {got[bad[0]]:#x} oracle {ref_tr[bad[0]]:#x}")
    ref = O.check(ref_tr, 2 * n_vars)
    st = t.status()
    assert np.array_equal(st, ref.status), f"{label}: status differs"
    assert np.array_equal(t.final(), ref.final), f"{label}: final differs"
    v = t.violations()
    assert v.total == ref.violations.size and np.array_equal(v.indices, ref.violations) and v.first == ref.first
    t.free()
    return ref


@pytest.mark.parametrize("ex", load_yaml("translation_examples.yaml"), ids=lambda e: e["name"])
def test_translation_worked_examples(ctx, ex):
    ids = {v: i for i, v in enumerate(ex["vars"])}
    co, de, nv, bo, bd = _components(ex, ids)
    all_ids = dict(ids)
    all_ids.update({v + "#": nv + i for v, i in ids.items()})
    t = gpu_translate(ctx, co, de, nv, bo, bd)
    assert list(t.events()) == list(parse_events(ex["translated"], all_ids))
    assert list(t.violations().indices) == ex["stuck"]
    t.free()


@pytest.mark.parametrize("seed", range(3))
def test_translation_small_canonical(ctx, seed):
    ct = gen.component_trace(5000, 64, seed)
    ref = assert_translation(ctx, ct.comp_off, ct.decls, ct.n_vars, label=f"small seed {seed}")
    assert ref.violations.size == 0  # Theorem 2 on well-declared programs


@pytest.mark.parametrize("n_comp,n_vars", [(1, 1), (3, 2), (4097, 8), (70_000, 1 << 12), (300_001, 1 << 20)])
def test_translation_shapes(ctx, n_comp, n_vars):
    ct = gen.component_trace(n_comp, n_vars, n_comp % 11, kmax=min(8, n_vars))
    assert_translation(ctx, ct.comp_off, ct.decls, ct.n_vars, label=f"{n_comp}x{n_vars}")


@pytest.mark.parametrize("n_comp,n_vars,kmax", [(50_000, 1 << 12, 14), (20_000, 1 << 10, 40)])
def test_translation_wide_components(ctx, n_comp, n_vars, kmax):
    """Components with up to 14 or 40 declarations: workgroups of 256 components whose
    declarations or events exceed what the fused emitter stages take the in-place path,
    the others the staged one (kmax 14 mixes both, kmax 40 is all in place)."""
    ct = gen.component_trace(n_comp, n_vars, 17 + kmax, kmax=kmax)
    ref = assert_translation(ctx, ct.comp_off, ct.decls, ct.n_vars, label=f"{n_comp}x{n_vars} kmax {kmax}")
    assert ref.violations.size == 0


def test_translation_empty_components(ctx):
    co = np.array([0, 0, 2, 2, 3, 3], np.uint64)
    de = np.array([decl("R", "GPU", 0), decl("W", "CPU", 1), decl("RW", "GPU", 1)], np.uint32)
    assert_translation(ctx, co, de, 2, label="empty components")


def test_translation_explicit_bodies(ctx):
    """Random (often ill-declared) explicit bodies: violations appear and must match."""
    ct = gen.component_trace(20_000, 128, 7)
    n_comp = ct.n_comp
    blen = gen.below(gen.draws(7, 200, 0, n_comp), 5)
    body_off = np.zeros(n_comp + 1, np.uint64)
    body_off[1:] = np.cumsum(blen)
    nb = int(body_off[-1])
    body = gen.plain_events(nb, 128, 7)
    ref = assert_translation(ctx, ct.comp_off, ct.decls, ct.n_vars, body_off, body, label="explicit bodies")
    assert ref.violations.size > 0


def test_translation_device_input_and_rerun(ctx):
    """Declarations resident on the device; re-running the translation reuses every buffer
    and gives the same bytes."""
    import torch
    from paper_1910_11110_amd import vcheck as V
    ct = gen.component_trace(200_000, 1 << 14, 3)
    co = torch.from_numpy(ct.comp_off.view(np.int64)).cuda()
    de = torch.from_numpy(ct.decls.view(np.int32)).cuda()
    torch.cuda.synchronize()
    t = V.translate(ctx, co, de, ct.n_vars, check=True)
    ctx.sync()
    ref_tr = O.translate(ct.comp_off, ct.decls, ct.n_vars)
    ref = O.check(ref_tr, 2 * ct.n_vars)
    for rep in range(3):
        say(f"[translate] device input run {rep}")
        assert np.array_equal(t.events(), ref_tr)
        assert np.array_equal(t.status(), ref.status)
        assert np.array_equal(t.final(), ref.final)
        V._check(V.lib().vc_translate_run(t.h))
        ctx.sync()
    t.free()


def test_translation_back_to_back_on_one_context(ctx):
    """Translations enqueued one after another on one context with a single wait at the
    end, then one of them run twice more without a wait between: the scan of the chunk
    counts runs on the context's second stream, forked after each translation's
    histogram pass and joined before its emitter, so no run may see another's counts."""
    import torch
    from paper_1910_11110_amd import vcheck as V
    cts = [gen.component_trace(300_000, 1 << 16, 11), gen.component_trace(120_000, 1 << 20, 12)]
    dev = [(torch.from_numpy(c.comp_off.view(np.int64)).cuda(), torch.from_numpy(c.decls.view(np.int32)).cuda())
           for c in cts]
    torch.cuda.synchronize()
    say("[translate] two translations, one wait")
    ts = [V.translate(ctx, co, de, c.n_vars, check=True) for (co, de), c in zip(dev, cts)]
    V._check(V.lib().vc_translate_run(ts[0].h))
    V._check(V.lib().vc_translate_run(ts[0].h))
    ctx.sync()
    for t, c in zip(ts, cts):
        ref_tr = O.translate(c.comp_off, c.decls, c.n_vars)
        ref = O.check(ref_tr, 2 * c.n_vars)
        assert np.array_equal(t.events(), ref_tr)
        assert np.array_equal(t.status(), ref.status)
        assert np.array_equal(t.final(), ref.final)
        v = t.violations()
        assert v.total == ref.violations.size and np.array_equal(v.indices, ref.violations)
        t.free()


def test_translation_malformed_declaration(ctx):
    from paper_1910_11110_amd import vcheck as V
    co = np.array([0, 2], np.uint64)
    de = np.array([decl("R", "CPU", 0), 3 << 24], np.uint32)  # mode 3 does not exist
    with pytest.raises(V.VCError) as ex:
        V.translate(ctx, co, de, 4)
    assert ex.value.code == V.VC_EINVAL and "index 1" in str(ex.value)


def test_translation_component_workload_full_size(ctx):
    """The component workload at full size: 2^23 components over 2^20 variables."""
    say("[translate] generating 2^23 components")
    ct = gen.component_trace(1 << 23, 1 << 20, 0)
    ref = assert_translation(ctx, ct.comp_off, ct.decls, ct.n_vars, label="full 2^23")
    assert ref.violations.size == 0


@pytest.mark.parametrize("n_comp,n_vars", [(5000, 64), (100_000, 1 << 14), (400_000, 1 << 20)])
def test_fused_and_unfused_check_agree(ctx, n_comp, n_vars):
    """Canonical bodies: the check fused into the emission equals translating first and
    checking the translated trace as a plain trace."""
    import os
    ct = gen.component_trace(n_comp, n_vars, 9)
    fused = gpu_translate(ctx, ct.comp_off, ct.decls, ct.n_vars)
    os.environ["VC_UNFUSED"] = "1"
    try:
        unfused = gpu_translate(ctx, ct.comp_off, ct.decls, ct.n_vars)
    finally:
        del os.environ["VC_UNFUSED"]
    assert np.array_equal(fused.events(), unfused.events())
    assert np.array_equal(fused.status(), unfused.status())
    assert np.array_equal(fused.final(), unfused.final())
    ref = O.check(O.translate(ct.comp_off, ct.decls, ct.n_vars), 2 * ct.n_vars)
    assert np.array_equal(fused.status(), ref.status) and np.array_equal(fused.final(), ref.final)
    fused.free()
    unfused.free()


@pytest.mark.parametrize("n_comp,n_vars,kmax", [(5000, 64, 8), (100_000, 1 << 14, 8), (300_001, 1 << 20, 8),
                                                (20_000, 1 << 10, 40)])
def test_device_and_host_sized_agree(ctx, n_comp, n_vars, kmax):
    """The fused translation finds its positions on the device (tiles look back for their
    base); with VC_HOST_SIZED it takes the per-component counts and the host-read length
    instead.  Same bytes, and the oracle's."""
    import os
    ct = gen.component_trace(n_comp, n_vars, 23 + kmax, kmax=kmax)
    say(f"[translate] device vs host sized {n_comp}x{n_vars} kmax {kmax}")
    dev = gpu_translate(ctx, ct.comp_off, ct.decls, ct.n_vars)
    os.environ["VC_HOST_SIZED"] = "1"
    try:
        host = gpu_translate(ctx, ct.comp_off, ct.decls, ct.n_vars)
    finally:
        del os.environ["VC_HOST_SIZED"]
    ref_tr = O.translate(ct.comp_off, ct.decls, ct.n_vars)
    ref = O.check(ref_tr, 2 * ct.n_vars)
    for t in (dev, host):
        assert t.info()[0] == ref_tr.size
        assert np.array_equal(t.events(), ref_tr)
        assert np.array_equal(t.status(), ref.status)
        assert np.array_equal(t.final(), ref.final)
        v = t.violations()
        assert v.total == ref.violations.size and v.first == ref.first
        t.free()


@pytest.mark.parametrize("host_sized", [False, True])
def test_translation_malformed_offsets_device(ctx, host_sized):
    """Component offsets in device memory that decrease are reported with the index of
    the component, on both ways of placing the events."""
    import os
    import torch
    from paper_1910_11110_amd import vcheck as V
    co = np.array([0, 3, 1, 4], np.uint64)  # component 1 ends before it starts
    de = np.array([decl("R", "CPU", 0), decl("W", "GPU", 1), decl("RW", "CPU", 2), decl("R", "GPU", 3)], np.uint32)
    tco = torch.from_numpy(co.view(np.int64)).cuda()
    tde = torch.from_numpy(de.view(np.int32)).cuda()
    torch.cuda.synchronize()
    if host_sized:
        os.environ["VC_HOST_SIZED"] = "1"
    try:
        with pytest.raises(V.VCError) as ex:
            t = V.translate(ctx, tco, tde, 4, check=True)
            ctx.sync()
            t.free()
    finally:
        os.environ.pop("VC_HOST_SIZED", None)
    assert "index 1" in str(ex.value)


def _with_repeat(n_comp, n_vars, seed, big=False):
    """A component program with one variable declared twice in one component (the
    declarations of a component must name distinct variables, Section 3.3); returns the
    inputs and the index the oracle reports."""
    ct = gen.component_trace(n_comp, n_vars, seed)
    co, de = ct.comp_off.copy(), ct.decls.copy()
    if big:
        # one component of 300 declarations (more than a wave tile stages) in the middle
        mid = n_comp // 2
        a = int(co[mid])
        extra = gen.pack_decls(np.arange(300) + 5, np.zeros(300, np.int64), np.zeros(300, np.int64))
        extra[290] = (extra[290] & ~np.uint32(0xFFFFFF)) | (extra[7] & np.uint32(0xFFFFFF))
        de = np.concatenate([de[:a], extra, de[a:]]).astype(np.uint32)
        co = np.concatenate([co[:mid + 1], co[mid + 1:] + np.uint64(300)]).astype(np.uint64)
        co = np.concatenate([co[:mid + 1], [co[mid] + np.uint64(300)], co[mid + 1:]]).astype(np.uint64)
    else:
        k = np.diff(co)
        c = int(np.nonzero(k >= 3)[0][len(np.nonzero(k >= 3)[0]) // 3])
        a = int(co[c])
        de[a + 2] = (de[a + 2] & ~np.uint32(0xFFFFFF)) | (de[a] & np.uint32(0xFFFFFF))
    with pytest.raises(O.OracleError) as ex:
        O.translate(co, de, n_vars)
    idx = int(str(ex.value).split("index ")[1])
    return co, de, idx


@pytest.mark.parametrize("where", ["host", "device", "device-host-sized", "device-unfused"])
@pytest.mark.parametrize("big", [False, True])
def test_translation_repeated_variable_rejected(ctx, where, big):
    """A variable declared twice in one component is malformed input: VC_EINVAL with the
    index of the second declaration, the oracle's, on every path (host validation, the
    wave emitter's look-back over the component, the serial pass of components too large
    to stage, and the per-component count kernel)."""
    import os
    import torch
    from paper_1910_11110_amd import vcheck as V
    co, de, idx = _with_repeat(20_000, 1 << 12, 5, big)
    say(f"[translate] repeated variable at {idx} ({where}, big={big})")
    env = {"device-host-sized": "VC_HOST_SIZED", "device-unfused": "VC_UNFUSED"}.get(where)
    if env:
        os.environ[env] = "1"
    try:
        with pytest.raises(V.VCError) as ex:
            if where == "host":
                V.translate(ctx, co, de, 1 << 12, check=True)
            else:
                tco = torch.from_numpy(co.view(np.int64)).cuda()
                tde = torch.from_numpy(de.view(np.int32)).cuda()
                torch.cuda.synchronize()
                t = V.translate(ctx, tco, tde, 1 << 12, check=True)
                ctx.sync()
                t.free()
    finally:
        if env:
            del os.environ[env]
    assert ex.value.code == V.VC_EINVAL and f"index {idx}" in str(ex.value), str(ex.value)


def test_translation_repeated_variable_minimal(ctx):
    """[W CPU x, R GPU x] in one component is rejected; the same declarations in two
    components translate and check as the oracle does."""
    from paper_1910_11110_amd import vcheck as V
    de = np.array([decl("W", "CPU", 0), decl("R", "GPU", 0)], np.uint32)
    with pytest.raises(V.VCError) as ex:
        V.translate(ctx, np.array([0, 2], np.uint64), de, 1, check=True)
    assert ex.value.code == V.VC_EINVAL and "index 1" in str(ex.value)
    assert_translation(ctx, np.array([0, 1, 2], np.uint64), de, 1, label="split over two components")
