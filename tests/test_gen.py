"""Seeded input generators: determinism, slicing and distribution sanity."""
import numpy as np

from paper_1910_11110_amd import gen


def test_splitmix_reference_values():
    # SplitMix64 with state 0: first outputs of the published generator
    base = np.uint64(0)
    with np.errstate(over="ignore"):
        z = gen._mix64(base + np.arange(1, 4, dtype=np.uint64) * gen.GAMMA)
    assert [int(x) for x in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_plain_events_deterministic_and_sliceable():
    a = gen.plain_events(5000, 64, 3)
    b = gen.plain_events(5000, 64, 3)
    assert np.array_equal(a, b)
    c = gen.plain_events(1000, 64, 3, start=2000)
    assert np.array_equal(a[2000:3000], c)
    assert not np.array_equal(a, gen.plain_events(5000, 64, 4))
    assert ((a >> 28) == 0).all() and ((a & 0xFFFFFF) < 64).all() and (((a >> 24) & 7) < 5).all()


def test_plain_events_law():
    e = gen.plain_events(1 << 20, 64, 0)
    op = np.bincount((e >> 24) & 7, minlength=5) / e.size
    assert np.allclose(op, 0.2, atol=0.005)
    assert abs(((e >> 27) & 1).mean() - 0.5) < 0.005
    v = np.bincount(e & 0xFFFFFF, minlength=64) / e.size
    assert np.allclose(v, 1 / 64, atol=0.002)


def test_component_trace_shape():
    ct = gen.component_trace(1 << 14, 1 << 12, 1)
    k = np.diff(ct.comp_off.astype(np.int64))
    assert k.min() >= 1 and k.max() <= 8 and abs(k.mean() - 4.5) < 0.1
    v = ct.decls & 0xFFFFFF
    for c in range(0, ct.n_comp, 97):
        seg = v[ct.comp_off[c]:ct.comp_off[c + 1]]
        assert len(set(seg.tolist())) == seg.size
    mode = (ct.decls >> 24) & 3
    frac = np.bincount(mode, minlength=3) / mode.size
    assert np.allclose(frac, [0.5, 0.3, 0.2], atol=0.02)
    side = (ct.decls >> 27) & 1
    for c in range(0, ct.n_comp, 101):
        seg = side[ct.comp_off[c]:ct.comp_off[c + 1]]
        assert (seg == seg[0]).all()
    # Zipf head: variable 0 is the most frequent
    cnt = np.bincount(v, minlength=1 << 12)
    assert cnt.argmax() == 0


def test_intervals_law():
    lo, hi = gen.intervals(1 << 16, 0)
    ln = hi.astype(np.int64) - lo
    assert ln.min() >= 1 and ln.max() <= 4096 and hi.max() <= (1 << 24)
    assert 400 < ln.mean() < 600


def test_trace_shapes():
    sh = gen.trace_shapes(4096, 0)
    lens = np.array([s.length for s in sh])
    nv = np.array([s.n_vars for s in sh])
    assert lens.min() >= 100 and lens.max() <= 1_000_000
    assert nv.min() >= 8 and nv.max() <= 65536
    assert 0.15 < np.mean([s.has_arrays for s in sh]) < 0.25
    assert sh[5] == gen.trace_shapes(10, 0)[5]
