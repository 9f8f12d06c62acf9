#!/usr/bin/env python3
"""Benchmark of the validity-status checker on one MI355X.

A step is one pass of the hot path over one batch of synthetic input.  The headline
workload is the VectorPU-style component trace (2^23 components over 2^20 variables,
Zipf(1.1) variables, R/W/RW = 0.5/0.3/0.2): declarations are translated into core
effects and the translated trace (~1.17e8 events) is checked in the same enqueue.
Inputs are generated on the host, copied to HBM once, and stay resident; the timed
region covers only device work.

Prints one JSON line.  By default the line also carries, under "also", the plain
single-trace workload at 2^28 events over 64 ids, the overlapping-array workload, the
workload with partial vectors created and destroyed during the trace, the batched
workload (4,096 traces) and the served workload (an open-loop Poisson replay), each
with its own roofline, oracle baseline and, for batched and served, the same traces
checked one after another by the per-trace path on the same GPU.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure (8 TB/s)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(label: str | None = None) -> str:
    """Digest of the kernel sources: all of them, or, for a kernel's profiling label, the
    headers and the source files that launch a kernel under that label (a change
    elsewhere leaves that kernel's counters valid)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1910_11110_amd", "csrc")
    files = sorted(os.listdir(d))
    if label is not None:
        key = f'"{label}"'.encode()
        srcs = []
        for f in files:
            if not f.endswith(".h"):
                with open(os.path.join(d, f), "rb") as fh:
                    if key in fh.read():
                        srcs.append(f)
        if srcs:
            files = sorted([f for f in files if f.endswith(".h")] + srcs)
    for f in files:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    when it was taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            t = json.load(f)
        e = t.get(workload, {}).get(kernel)
        if e and e.get("source_digest") == source_digest(kernel):
            return e["bytes_per_launch"]
    except Exception:
        return None
    return None


def host_info() -> dict:
    """The host the oracle is timed on: CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def pool_threads() -> int:
    """Threads for the all-core oracle timing: every usable core, at most 16 (the GPU
    box's CPU share for one GPU)."""
    return max(1, min(16, host_info()["nproc"] or 1))


class Timer:
    """HIP events on the stream the library launches on."""

    def __init__(self, stream):
        import torch
        self.torch = torch
        self.stream = stream

    def __enter__(self):
        self.a = self.torch.cuda.Event(enable_timing=True)
        self.b = self.torch.cuda.Event(enable_timing=True)
        self.a.record(self.stream)
        return self

    def __exit__(self, *exc):
        self.b.record(self.stream)
        self.b.synchronize()
        self.ms = self.a.elapsed_time(self.b)


def _median_rate(units, fn, runs=3):
    times = []
    for _ in range(runs):
        a = time.perf_counter()
        fn()
        times.append(time.perf_counter() - a)
    return units / float(np.median(times))


# ------------------------------------------------------------------------------------------
# workloads: each returns step(), the units of a step, the algorithmic bytes of a step
# (the method's inputs read once and outputs written once), the oracle timing and config
# ------------------------------------------------------------------------------------------
def wl_components(args, V, ctx, stream):
    import torch
    from paper_1910_11110_amd import gen
    n_comp, n_vars = 1 << args.comp_log2, 1 << 20
    log(f"[bench] components: generating {n_comp} components over {n_vars} variables")
    ct = gen.component_trace(n_comp, n_vars, args.seed)
    co = torch.from_numpy(ct.comp_off.view(np.int64)).cuda()
    de = torch.from_numpy(ct.decls.view(np.int32)).cuda()
    torch.cuda.synchronize()
    t = V.translate(ctx, co, de, n_vars, check=True)
    ctx.sync()
    n_ev, _ = t.info()
    viol = t.violations().total

    def step():
        t.rerun()

    def bytes_alg():
        # declarations (4 B) and component offsets (8 B) read once; the translated trace
        # (4 B), one status byte per event, the violation indices and the final statuses
        # of real and abstract variables written once
        return 4 * ct.decls.size + 8 * (n_comp + 1) + 4 * n_ev + n_ev + 4 * viol + 2 * n_vars

    def cpu_sample():
        from oracle import oracle as O

        def run():
            tr = O.translate(ct.comp_off, ct.decls, n_vars)
            O.check(tr, 2 * n_vars)
        return _median_rate(n_ev, run), "oracle translate + check of the full workload, median of 3 runs", None

    nd = int(ct.decls.size)
    # each kernel's own minimum traffic: its inputs read once, its outputs written once
    own_io = {
        "bucket_hist": (4 * nd + 4 * (nd // 64), nd, "declaration"),      # words; chunk event counts
        "partition": (12 * nd, nd, "declaration"),                       # words in; words, destinations out
        "bucket_scan": (5 * nd + n_vars, nd, "declaration"),             # words in, pre-status out, final
        "translate_emit_wave": (9 * nd + 8 * (n_comp + 1) + 5 * n_ev, n_ev, "translated event"),
    }
    cfg = {"workload": f"components-2^{args.comp_log2}", "n_components": n_comp, "n_vars": n_vars,
           "n_declarations": nd, "n_events": int(n_ev), "violations": int(viol)}
    return dict(step=step, units=n_ev, unit="translated event", bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg,
                keep=(t, co, de), own_io=own_io)


def wl_plain(args, V, ctx, stream, n=None, n_ids=64):
    import torch
    from paper_1910_11110_amd import gen
    n = n or (1 << args.plain_log2)
    log(f"[bench] plain: generating {n} events over {n_ids} ids")
    e = gen.plain_events(n, n_ids, args.seed)
    te = torch.from_numpy(e.view(np.int32)).cuda()
    torch.cuda.synchronize()
    t = V.Trace.load(ctx, te, n_ids)
    t.check()
    ctx.sync()
    viol = t.violations().total

    def step():
        t.check()

    def bytes_alg():
        # events in (4 B), status bytes out (1 B), violation indices, final table
        return 4 * n + n + 4 * viol + n_ids

    def cpu_sample():
        from oracle import oracle as O
        m = min(n, 1 << 27)
        return (_median_rate(m, lambda: O.check(e[:m], n_ids)),
                f"oracle check of the first {m} events, median of 3 runs", None)

    own_io = {
        "small_check": (5 * n + 4 * viol + n_ids, n, "event"),
        "bucket_hist": (4 * n, n, "event"),
        "partition": (12 * n, n, "event"),
        "bucket_scan": (5 * n + n_ids, n, "event"),
        "replay_status": (6 * n + 4 * viol, n, "event"),
    }
    cfg = {"workload": f"plain-{n}x{n_ids}", "n_events": n, "n_ids": n_ids, "violations": int(viol)}
    return dict(step=step, units=n, unit="event", bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(t, te),
                own_io=own_io)


def wl_overlap(args, V, ctx, stream):
    import torch
    from paper_1910_11110_amd import gen
    n_arr, n = 1 << 16, 1 << 24
    lo, hi = gen.intervals(n_arr, args.seed)
    e = gen.plain_events(n, n_arr, args.seed)
    te = torch.from_numpy(e.view(np.int32)).cuda()
    torch.cuda.synchronize()
    t = V.Trace.load(ctx, te, n_arr)
    a = time.perf_counter()
    t.set_arrays(lo, hi)
    sweep_s = time.perf_counter() - a
    t.check()
    ctx.sync()
    viol = t.violations().total

    def step():
        t.check()

    def bytes_alg():
        return 4 * n + n + 4 * viol + n_arr + 8 * n_arr

    def cpu_sample():
        from oracle import oracle as O
        sets = O.overlap_sets(lo, hi)
        return (_median_rate(n, lambda: O.check_overlap(e, lo, hi, sets=sets)),
                "oracle overlap check of the full workload (overlap sets precomputed), median of 3", None)

    cfg = {"workload": "overlap-2^16-arrays-2^24-events", "n_events": n, "n_arrays": n_arr, "violations": int(viol),
           "interval_sweep_ms_incl_host": round(sweep_s * 1e3, 3)}
    return dict(step=step, units=n, unit="event", bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(t, te))


def wl_dynamic(args, V, ctx, stream):
    """Partial vectors created and destroyed during the trace: 2^24 events over 2^10
    vectors (tiling a 2^24-element address space) and 64,512 partial vectors (lengths
    log-uniform in [1, 4096], a quarter live from the start, half destroyed)."""
    from paper_1910_11110_amd import gen
    n, nv = 1 << 24, 1 << 10
    log(f"[bench] dynamic: generating {n} events over {1 << 16} arrays")
    d = gen.dynamic_trace(n, nv, (1 << 16) - nv, args.seed)
    t = V.Trace.load(ctx, d.events, d.lo.size, lifetimes=True)
    t.set_dynamic_arrays(d.lo, d.hi, d.mother)
    t.check()
    ctx.sync()
    viol = t.violations().total
    n_ids = int(d.lo.size)

    def step():
        t.check()

    def bytes_alg():
        # events in, status bytes out, violation indices, final table; intervals and
        # mothers read once
        return 4 * n + n + 4 * viol + n_ids + 12 * n_ids

    def cpu_sample():
        from oracle import oracle as O
        sets = O.overlap_sets(d.lo, d.hi)
        return (_median_rate(n, lambda: O.check_dynamic(d.events, d.lo, d.hi, d.mother, sets=sets)),
                "oracle dynamic check of the full workload (overlap sets precomputed), median of 3", None)

    cfg = {"workload": "dynamic-2^16-arrays-2^24-events", "n_events": n, "n_vectors": nv, "n_arrays": n_ids,
           "creates": int(((d.events >> 24) & 7 == 6).sum()), "destroys": int(((d.events >> 24) & 7 == 7).sum()),
           "violations": int(viol)}
    return dict(step=step, units=n, unit="event", bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(t, d),
                multi_pass=("sort_pass", "hist"))


def wl_spaces(args, V, ctx, stream):
    """Four memory spaces: 2^26 events over 2^20 variables, op uniform over {r, w, copy,
    Noop}, locations uniform."""
    import torch
    from paper_1910_11110_amd import gen
    n, n_ids, k = 1 << 26, 1 << 20, 4
    log(f"[bench] spaces: generating {n} events over {n_ids} ids, k = {k}")
    e = gen.space_events(n, n_ids, k, args.seed)
    te = torch.from_numpy(e.view(np.int32)).cuda()
    torch.cuda.synchronize()
    t = V.Trace.load_spaces(ctx, te, n_ids, k)
    t.check()
    ctx.sync()
    viol = t.violations().total

    def step():
        t.check()

    def bytes_alg():
        # events in (4 B), uint16 statuses out, violation indices, final codes
        return 4 * n + 2 * n + 4 * viol + n_ids

    def cpu_sample():
        from oracle import oracle as O
        m = 1 << 25
        return (_median_rate(m, lambda: O.check_spaces(e[:m], n_ids, k)),
                f"oracle check of the first {m} events, median of 3 runs", None)

    cfg = {"workload": f"spaces-k{k}-2^26x2^20", "n_events": n, "n_ids": n_ids, "k": k, "violations": int(viol)}
    return dict(step=step, units=n, unit="event", bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(t, te),
                multi_pass=("sort_pass", "hist"))


def wl_declared(args, V, ctx, stream):
    """Well-declaredness of 2^20 components over 2^16 arrays (lengths log-uniform in
    [1, 64] in a 2^22-element space), bodies of explicit element accesses, 5 % of the
    components altered, checked against the declarations extended for overlaps."""
    import torch
    from paper_1910_11110_amd import gen
    n_comp, n_vars = 1 << 20, 1 << 16
    log(f"[bench] declared: generating {n_comp} components over {n_vars} arrays")
    p = gen.declared_program(n_comp, n_vars, args.seed, arrays=True, space=1 << 22, max_len=64)
    dev = [torch.from_numpy(a.view(np.int64 if a.dtype == np.uint64 else np.int32)).cuda()
           for a in (p.comp_off, p.decls, p.body_off, p.body, p.idx)]
    torch.cuda.synchronize()
    t = V.check_declared(ctx, dev[0], dev[1], n_vars, dev[2], dev[3], dev[4], p.lo, p.hi, extend=True)
    ctx.sync()
    ill = t.violations().total
    nb, nd = int(p.body.size), int(p.decls.size)

    def step():
        t.check()

    def bytes_alg():
        # offsets, declarations, body words and element indices read once, intervals
        # once; one verdict byte per component and the ill-declared indices written
        return 16 * (n_comp + 1) + 4 * nd + 8 * nb + 8 * n_vars + n_comp + 4 * ill

    def cpu_sample():
        from oracle import oracle as O
        sets = O.overlap_sets(p.lo, p.hi)
        return (_median_rate(nb, lambda: O.check_declared(p.comp_off, p.decls, n_vars, p.body_off, p.body, p.idx,
                                                           p.lo, p.hi, extend=True, sets=sets)),
                "oracle well-declaredness check of the full workload (overlap sets precomputed), median of 3 "
                "(body events/s)", None)

    cfg = {"workload": "declared-2^20-components-2^16-arrays", "n_components": n_comp, "n_arrays": n_vars,
           "n_declarations": nd, "n_body_events": nb, "ill_declared": int(ill), "extend": True}
    return dict(step=step, units=nb, unit="body event", bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg,
                keep=(t, dev, p))


def wl_programs(args, V, ctx, stream):
    """Structured programs: 2^20 programs over 16 variables each, drawn from 4,096 random
    templates of up to 64 words (While and If on isValid, remIsValid and choice
    conditions, nested up to 4 deep), own choice words and initial statuses, fuel 4096
    reductions."""
    from paper_1910_11110_amd import gen
    n_prog, n_vars, fuel = 1 << 20, 16, 1 << 12
    log(f"[bench] programs: generating {n_prog} programs")
    P = gen.structured_programs(n_prog, n_vars, args.seed)
    g = V.Programs(ctx, P.prog_off, P.words, n_vars, P.choice, P.init, fuel)
    steps = int(g.read()[0].sum())

    def step():
        g.run()

    def bytes_alg():
        # program words, offsets, choice words and initial statuses read once; five
        # counters and the final statuses of every program written once
        return 4 * int(P.words.size) + 8 * (n_prog + 1) + 8 * n_prog + n_vars * n_prog + 33 * n_prog + n_vars * n_prog

    def cpu_sample():
        from oracle import oracle as O
        m = 1 << 17
        po = P.prog_off[:m + 1]
        return (_median_rate(int(O.run_programs(po, P.words, n_vars, P.choice[:m], P.init[:m * n_vars],
                                                fuel).steps.sum()),
                             lambda: O.run_programs(po, P.words, n_vars, P.choice[:m], P.init[:m * n_vars], fuel)),
                f"oracle run of the first {m} programs, median of 3 (reductions/s)", None)

    cfg = {"workload": "programs-2^20x16-fuel-4096", "n_programs": n_prog, "n_vars": n_vars, "fuel": fuel,
           "n_words": int(P.words.size), "reductions": steps}
    return dict(step=step, units=steps, unit="reduction", bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg,
                keep=(g, P))


def _oracle_job(inp, sets):
    from oracle import oracle as O
    ev, nv, lo, hi = inp
    if lo is None:
        O.check(ev, nv)
    else:
        O.check_overlap(ev, lo, hi, sets=sets)


def _oracle_traces(inputs, budget_events):
    """The oracle over the first traces of `inputs` ((events, n_ids, lo, hi)) up to about
    budget_events events, on one host core and then trace-parallel on every usable core.
    Overlap sets are computed before the clock starts: only the evaluation is timed."""
    from oracle import oracle as O
    take, m = [], 0
    for inp in inputs:
        if m >= budget_events:
            break
        take.append(inp)
        m += inp[0].size
    sets = [None if lo is None else O.overlap_sets(lo, hi) for _e, _n, lo, hi in take]
    a = time.perf_counter()
    for inp, s in zip(take, sets):
        _oracle_job(inp, s)
    one = m / (time.perf_counter() - a)
    k = pool_threads()
    a = time.perf_counter()
    with cf.ThreadPoolExecutor(k) as ex:
        list(ex.map(lambda js: _oracle_job(*js), zip(take, sets)))
    allc = m / (time.perf_counter() - a)
    return one, allc, k, len(take), m


def _sequential_per_trace(V, ctx, traces, units):
    """The same traces checked one after another by the per-trace path (vc_check on each
    resident trace, all enqueued on the context's stream, one wait at the end)."""
    best = None
    for _ in range(3):
        ctx.sync()
        a = time.perf_counter()
        for t in traces:
            t.check()
        ctx.sync()
        s = time.perf_counter() - a
        best = s if best is None else min(best, s)
    return {"value": round(units / best, 1), "unit": "events/s", "ms": round(best * 1e3, 3),
            "how": "vc_check on every trace in turn (inputs resident), one sync at the end; best of 3"}


def wl_batched(args, V, ctx, stream):
    """4,096 independent traces (lengths log-uniform in [100, 10^6], variables log-uniform
    in [8, 65,536], 20 % with array intervals), loaded once; a step is one batched check
    of all of them (one pipeline, replayed as a HIP graph)."""
    from paper_1910_11110_amd import gen
    n_tr = 4096
    log(f"[bench] batched: generating {n_tr} traces")
    shapes = gen.trace_shapes(n_tr, args.seed)
    traces, inputs = [], []
    for sh in shapes:
        ev, lo, hi = gen.trace_inputs(sh)
        t = V.Trace.load(ctx, ev, sh.n_vars)
        if lo is not None:
            t.set_arrays(lo, hi)
        traces.append(t)
        inputs.append((ev, sh.n_vars, lo, hi))
    n = sum(sh.length for sh in shapes)
    log(f"[bench] batched: {n} events; first batched check")
    V.batch_check(ctx, traces)
    ctx.sync()
    viol = sum(t.violations().total for t in traces)
    ids = sum(sh.n_vars for sh in shapes)

    def step():
        V.batch_check(ctx, traces)

    def bytes_alg():
        return 4 * n + n + 4 * viol + ids

    def cpu_sample():
        one, allc, k, nt, m = _oracle_traces(inputs, 1 << 25)
        return one, f"oracle check of the first {nt} traces ({m} events), one run, overlap sets precomputed", \
            {"value": round(allc, 1), "threads": k}

    def extra():
        log("[bench] batched: the same traces through the per-trace path, one after another")
        return {"sequential_per_trace": _sequential_per_trace(V, ctx, traces, n)}

    cfg = {"workload": "batched-4096-traces", "n_traces": n_tr, "n_events": n,
           "with_arrays": sum(1 for sh in shapes if sh.has_arrays), "violations": int(viol)}
    return dict(step=step, units=n, unit="event", bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg,
                keep=(traces, inputs), extra=extra, multi_pass=("sort_pass", "hist"))


# ------------------------------------------------------------------------------------------
# served: open-loop Poisson replay
# ------------------------------------------------------------------------------------------
def _served_pool(seed, n_pool):
    from paper_1910_11110_amd import gen
    shapes = gen.trace_shapes(n_pool, seed + 100)
    pool = []
    for sh in shapes:
        ev, lo, hi = gen.trace_inputs(sh)
        pool.append((ev, sh.n_vars, lo, hi, np.empty(ev.size, np.uint8)))
    return pool


def _replay(V, ctx, pool, arrivals, budget, chunk, label):
    """Opens one stream per arrival (pool trace i % len(pool)) at its arrival time, submits
    all its chunks then (a stream's chunks run in order, one at a time), and closes it
    when its last chunk has completed.  Returns latencies and throughput."""
    srv = V.Server(ctx, budget)
    n_arr = arrivals.size
    open_ = {}   # stream -> [pool index, chunks left, arrival (server clock), last done]
    chunk_lat, trace_lat = [], []
    done_events, i, viol = 0, 0, 0
    t0 = srv.now()
    last_done = t0
    deadline = t0 + float(arrivals[-1] if n_arr else 0.0) + 120.0
    while i < n_arr or open_:
        now = srv.now()
        while i < n_arr and t0 + arrivals[i] <= now:
            ev, nv, lo, hi, out = pool[i % len(pool)]
            s = srv.open(nv, lo, hi)
            k = 0
            for a in range(0, ev.size, chunk):
                srv.submit(s, ev[a:a + chunk], out[a:a + chunk])
                k += 1
            open_[s] = [i % len(pool), k, t0 + float(arrivals[i]), 0.0]
            i += 1
        cs = srv.poll()
        for c in cs:
            if c.status != 0:
                raise RuntimeError(f"{label}: chunk {c.chunk} failed with {c.status}")
            chunk_lat.append(c.t_done - c.t_submit)
            done_events += c.n_events
            viol += c.n_violations
            st = open_[c.stream]
            st[1] -= 1
            st[3] = max(st[3], c.t_done)
            last_done = max(last_done, c.t_done)
        for s in [s for s, st in open_.items() if st[1] == 0]:
            st = open_.pop(s)
            trace_lat.append(st[3] - st[2])
            srv.close_stream(s, pool[st[0]][1])
        if not cs:
            if srv.now() > deadline:
                raise RuntimeError(f"{label}: completions stalled")
            time.sleep(0.0002)
    srv.close()
    span = last_done - t0
    cl = np.sort(np.asarray(chunk_lat)) * 1e3
    tl = np.sort(np.asarray(trace_lat)) * 1e3

    def pct(a, q):
        return round(float(a[min(a.size - 1, (a.size * q) // 100)]), 3) if a.size else None
    return {"traces": int(n_arr), "chunks": int(cl.size), "events": int(done_events), "violations": int(viol),
            "span_s": round(span, 3), "sustained_events_per_s": round(done_events / span, 1) if span > 0 else None,
            "chunk_latency_ms": {"p50": pct(cl, 50), "p99": pct(cl, 99), "max": round(float(cl[-1]), 3)},
            "trace_latency_ms": {"p50": pct(tl, 50), "p99": pct(tl, 99), "max": round(float(tl[-1]), 3)}}


def served_report(args, V, ctx):
    """Served workload: Poisson arrivals of traces with the batched workload's shapes, each
    split into 2^16-event chunks, its status table resident on the device between chunks;
    admission by a 64 GB budget (and, in a second replay, by a 64 MB budget that binds)."""
    from paper_1910_11110_amd import gen
    chunk = 1 << 16
    log(f"[bench] served: generating a pool of {args.served_pool} traces")
    pool = _served_pool(args.seed, args.served_pool)
    pool_events = sum(p[0].size for p in pool)
    arrivals = gen.poisson_arrivals(args.served_rate, args.served_seconds, args.seed)
    offered = float(np.mean([p[0].size for p in pool])) * args.served_rate
    log(f"[bench] served: replay of {arrivals.size} arrivals over {args.served_seconds} s at 64 GB")
    main = _replay(V, ctx, pool, arrivals, 64 << 30, chunk, "64 GB replay")
    log("[bench] served: capacity (the whole pool arriving at once)")
    cap = _replay(V, ctx, pool, np.zeros(len(pool)), 64 << 30, chunk, "capacity")
    small_s = min(5.0, args.served_seconds)
    arr2 = arrivals[arrivals < small_s]
    log(f"[bench] served: replay of {arr2.size} arrivals over {small_s} s at 64 MB")
    tight = _replay(V, ctx, pool, arr2, 64 << 20, chunk, "64 MB replay")
    log("[bench] served: the pool through the per-trace path, one after another")
    seq = None
    for _ in range(2):
        a = time.perf_counter()
        for ev, nv, lo, hi, out in pool:
            t = V.Trace.load(ctx, ev, nv)
            if lo is not None:
                t.set_arrays(lo, hi)
            t.check()
            ctx.sync()
            t.status()
            t.free()
        s = time.perf_counter() - a
        seq = s if seq is None else min(seq, s)
    cpu = None
    if not args.no_cpu_baseline:
        one, allc, k, nt, m = _oracle_traces([p[:4] for p in pool], 1 << 25)
        cpu = {"value": round(one, 1), "unit": "events/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle check of the first {nt} pool traces ({m} events), overlap sets precomputed",
               "host": host_info(), "all_cores": {"value": round(allc, 1), "threads": k}}
    rec = {
        "config": {"workload": "served-poisson", "rate_traces_per_s": args.served_rate,
                   "duration_s": args.served_seconds, "chunk_events": chunk, "budget_bytes": 64 << 30,
                   "trace_pool": len(pool), "pool_events": int(pool_events),
                   "shapes": "lengths log-uniform [100, 1e6], variables log-uniform [8, 65536], 20% with arrays",
                   "offered_events_per_s": round(offered, 1)},
        "value": main["sustained_events_per_s"], "unit": "events/s",
        "replay": main,
        "capacity": cap,
        "tight_budget_64MB": tight,
        "sequential_per_trace": {"value": round(pool_events / seq, 1), "unit": "events/s", "ms": round(seq * 1e3, 3),
                                 "how": "per pool trace: load from host, set arrays, vc_check, sync, read the "
                                        "status bytes, free; best of 2"},
        "cpu_baseline": cpu,
        "note": "latencies are submit-to-completion on the server clock, queueing included; a trace's latency "
                "runs from its arrival to its last chunk's completion; the replay includes the chunks' copies "
                "from host memory and the status bytes' copies back",
    }
    return rec


def copy_probe(torch, n_words=1 << 28):
    """One plain elementwise kernel of known traffic (reads and writes 4 * n_words bytes),
    launched before the workload so that a hardware-counter run of this script also
    holds the calibration of FETCH_SIZE / WRITE_SIZE against known bytes."""
    x = torch.ones(n_words, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y
    return 4 * n_words


WORKLOADS = {"components": wl_components, "plain-large": wl_plain,
             "plain-wide": lambda a, V, c, s: wl_plain(a, V, c, s, n=1 << 26, n_ids=1 << 20),
             "plain-small": lambda a, V, c, s: wl_plain(a, V, c, s, n=10_000), "overlap": wl_overlap,
             "batched": wl_batched, "dynamic": wl_dynamic, "spaces": wl_spaces, "declared": wl_declared,
             "programs": wl_programs}


def measure(name, args, V, ctx, stream, steps, warmup, cpu=True):
    """Runs `steps` timed steps of a workload after `warmup` untimed ones and returns its
    record: throughput, the roofline of its dominant kernel, the whole step's fraction of
    peak, per-kernel times and the oracle baseline."""
    import torch
    w = WORKLOADS[name](args, V, ctx, stream)
    for _ in range(warmup):
        w["step"]()
    ctx.sync()
    torch.cuda.synchronize()
    # timed region: exactly `steps` steps, synchronized on both sides
    with Timer(stream) as tm:
        for _ in range(steps):
            w["step"]()
    ctx.sync()
    ms_step = tm.ms / steps
    value = w["units"] / (ms_step / 1e3)

    # per-kernel durations: the same steps again with event pairs around each kernel
    ctx.profile(True)
    ctx.profile_reset()
    for _ in range(steps):
        w["step"]()
    prof = ctx.profile_read()
    ctx.profile(False)
    kernels = {k: {"ms_per_launch": ms / max(n, 1), "launches_per_step": n / steps, "ms_per_step": ms / steps}
               for k, (ms, n) in prof.items()}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"]) if kernels else None
    alg_step = w["bytes_alg"]()
    per_unit = alg_step / w["units"]
    roof = None
    if dom:
        d = kernels[dom]
        # units one launch of the dominant kernel processes: every unit for a kernel that
        # passes over the whole input on each launch (sort passes), else the step's units
        # spread over its launches
        multi = any(dom.startswith(p) for p in w.get("multi_pass", ()))
        upl = w["units"] if multi or d["launches_per_step"] <= 1 else w["units"] / d["launches_per_step"]
        achieved = per_unit * upl / (d["ms_per_launch"] / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom, name),
                "bytes_per_unit": round(per_unit, 4), "unit_of_work": w["unit"], "units_per_launch": int(upl),
                "ms_per_launch": round(d["ms_per_launch"], 4),
                "basis": "the path's algorithmic bytes per unit (inputs read once, outputs written once) x the "
                         "units one launch processes / the kernel's mean launch time (HIP events)"}
    # each kernel's own minimum I/O (intermediates of the sort included), for comparison
    own = {}
    for k, (b, units, unit) in w.get("own_io", {}).items():
        if k in kernels and kernels[k]["ms_per_launch"] > 0:
            gbs = b / (kernels[k]["ms_per_launch"] / 1e3) / 1e9
            own[k] = {"bytes_per_launch": int(b), "units_per_launch": int(units), "unit": unit,
                      "achieved_GBs": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    pipeline = {"algorithmic_bytes_per_step": int(alg_step), "bytes_per_unit": round(per_unit, 4),
                "achieved_GBs": round(alg_step / (ms_step / 1e3) / 1e9, 2),
                "frac": round(alg_step / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    cpu_rec = None
    if cpu:
        log(f"[bench] {name}: timing the oracle on the host")
        v, sample, allc = w["cpu"]()
        cpu_rec = {"value": round(v, 1), "unit": "events/s", "cores": 1, "kind": "oracle", "sample": sample,
                   "host": host_info()}
        if allc:
            cpu_rec["all_cores"] = allc
    rec = {"config": w["config"], "value": round(value, 1), "unit": "events/s", "steps": steps, "warmup": warmup,
           "ms_per_step": round(ms_step, 4), "roofline": roof, "pipeline_roofline": pipeline, "cpu_baseline": cpu_rec,
           "kernel_own_io": own,
           "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in kernels.items()}}
    if "extra" in w:
        rec.update(w["extra"]())
    del w
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="components", choices=sorted(WORKLOADS) + ["served"])
    ap.add_argument("--also", default="plain-large,overlap,dynamic,spaces,declared,programs,batched,served",
                    help="workloads reported beside the headline one (comma separated; empty for none)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--comp-log2", type=int, default=23)
    ap.add_argument("--plain-log2", type=int, default=28)
    ap.add_argument("--served-rate", type=float, default=2000.0)
    ap.add_argument("--served-seconds", type=float, default=15.0)
    ap.add_argument("--served-pool", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="launch one 1 GiB elementwise kernel first (calibrates hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the checker is a single-GPU path); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1910_11110_amd import vcheck as V
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = V.Context(0, stream)
    if args.copy_probe:
        log(f"[bench] copy probe: {copy_probe(torch)} bytes read and written")
    cpu = not args.no_cpu_baseline
    if args.workload == "served":
        head = served_report(args, V, ctx)
        head.update(steps=1, warmup=0, ms_per_step=None, roofline=None)
    else:
        head = measure(args.workload, args, V, ctx, stream, args.steps, args.warmup, cpu)
    also = {}
    for name in [x for x in args.also.split(",") if x and x != args.workload]:
        if name == "served":
            also[name] = served_report(args, V, ctx)
        else:
            also[name] = measure(name, args, V, ctx, stream, args.steps, args.warmup, cpu)
    out = {
        "metric": "trace events checked/sec (bit-exact)",
        "value": head["value"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": head["warmup"],
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
    }
    for k, v in head.items():
        if k not in out and k not in ("unit",):
            out[k] = v
    out["also"] = also
    out["source_digest"] = source_digest()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
