#!/usr/bin/env python3
"""Benchmark of the validity-status checker on one MI355X.

A step is one pass of the hot path over one batch of synthetic input.  The default
workload is the VectorPU-style component trace (2^23 components over 2^20
variables, Zipf(1.1) variables, R/W/RW = 0.5/0.3/0.2): declarations are
translated into core effects and the translated trace (~1.17e8 events) is checked
in the same enqueue.  Inputs are generated on the host, copied to HBM once, and
stay resident; the timed region covers only device work (plus the one host-visible
size read-back the translation does).

Prints one JSON line.  Extra workloads (--workload) report the same schema.
"""
from __future__ import annotations

import argparse
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


def source_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1910_11110_amd", "csrc")
    for f in sorted(os.listdir(d)):
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
        if e and e.get("source_digest") == source_digest():
            return e["bytes_per_launch"]
    except Exception:
        return None
    return None


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


# ------------------------------------------------------------------------------------------
# workloads
# ------------------------------------------------------------------------------------------
def wl_components(args, V, ctx, stream):
    import torch
    from paper_1910_11110_amd import gen
    n_comp, n_vars = 1 << args.comp_log2, 1 << 20
    log(f"[bench] generating {n_comp} components over {n_vars} variables")
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
        # read declarations and offsets once; write the translated trace, one status
        # byte per event, the violation indices and the final statuses
        return 4 * ct.decls.size + 8 * (n_comp + 1) + 4 * n_ev + n_ev + 4 * viol + 2 * n_vars

    def cpu_sample():
        from oracle import oracle as O
        times = []
        for _ in range(3):
            a = time.perf_counter()
            tr = O.translate(ct.comp_off, ct.decls, n_vars)
            O.check(tr, 2 * n_vars)
            times.append(time.perf_counter() - a)
        return n_ev / float(np.median(times)), f"oracle translate+check of the full workload, median of 3 runs"

    nd = int(ct.decls.size)
    # each kernel's own algorithmic traffic: its inputs read once, its outputs written once
    # (unit: declarations for the declaration passes, translated events for the emitter)
    kernel_bytes = {
        "bucket_hist": (4 * nd + 4 * (nd // 64), nd, "declaration"),      # words; chunk event counts
        "partition": (12 * nd, nd, "declaration"),                       # words in; words, destinations out
        "bucket_scan": (5 * nd + n_vars, nd, "declaration"),             # words in, pre-status out, final
        # declarations, their destinations and gathered pre-statuses, offsets; events and status bytes out
        "translate_emit_wave": (9 * nd + 8 * (n_comp + 1) + 5 * n_ev, n_ev, "translated event"),
    }
    cfg = {"workload": f"components-2^{args.comp_log2}", "n_components": n_comp, "n_vars": n_vars,
           "n_declarations": nd, "n_events": int(n_ev), "violations": int(viol)}
    return dict(step=step, units=n_ev, bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(t, co, de),
                per_unit=lambda: bytes_alg() / n_ev, kernel_bytes=kernel_bytes)


def wl_plain(args, V, ctx, stream, n=None, n_ids=64):
    import torch
    from paper_1910_11110_amd import gen
    n = n or (1 << args.plain_log2)
    log(f"[bench] generating {n} plain events over {n_ids} ids")
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
        return 4 * n + n + 4 * viol + n_ids

    def cpu_sample():
        from oracle import oracle as O
        m = min(n, 1 << 27)
        times = []
        for _ in range(3):
            a = time.perf_counter()
            O.check(e[:m], n_ids)
            times.append(time.perf_counter() - a)
        return m / float(np.median(times)), f"oracle check of the first {m} events, median of 3 runs"

    kernel_bytes = {
        "small_check": (5 * n + 4 * viol + n_ids, n, "event"),              # events in, status out, violations
        "bucket_hist": (4 * n, n, "event"),
        "partition": (12 * n, n, "event"),                                  # words in; words, destinations out
        "bucket_scan": (5 * n + n_ids, n, "event"),
        "replay_status": (6 * n + 4 * viol, n, "event"),                    # destinations, gathered byte, status, violations
    }
    cfg = {"workload": f"plain-{n}x{n_ids}", "n_events": n, "n_ids": n_ids, "violations": int(viol)}
    return dict(step=step, units=n, bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(t, te),
                per_unit=lambda: bytes_alg() / n, kernel_bytes=kernel_bytes)


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
        return 4 * n + n + 4 * viol + n_arr

    def cpu_sample():
        from oracle import oracle as O
        sets = O.overlap_sets(lo, hi)
        times = []
        for _ in range(3):
            a = time.perf_counter()
            O.check_overlap(e, lo, hi, sets=sets)
            times.append(time.perf_counter() - a)
        return n / float(np.median(times)), "oracle overlap check of the full workload (sets precomputed), median of 3"

    cfg = {"workload": "overlap-2^16-arrays-2^24-events", "n_events": n, "n_arrays": n_arr, "violations": int(viol),
           "interval_sweep_ms_incl_host": round(sweep_s * 1e3, 3)}
    return dict(step=step, units=n, bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(t, te),
                per_unit=lambda: bytes_alg() / n)


def _oracle_sample(inputs, budget_events):
    """events/s of the oracle over the first traces of `inputs` ((events, n_ids, lo, hi))
    up to about budget_events events; and how many traces and events that was"""
    from oracle import oracle as O
    take, m = [], 0
    for inp in inputs:
        if m >= budget_events:
            break
        take.append(inp)
        m += inp[0].size
    a = time.perf_counter()
    for ev, nv, lo, hi in take:
        if lo is None:
            O.check(ev, nv)
        else:
            O.check_overlap(ev, lo, hi)
    return m / (time.perf_counter() - a), len(take), m


def wl_batched(args, V, ctx, stream):
    """4,096 independent traces (lengths log-uniform in [100, 10^6], variables log-uniform
    in [8, 65,536], 20 % with array intervals), loaded once; a step is one batched check
    of all of them (one pipeline, replayed as a HIP graph)."""
    from paper_1910_11110_amd import gen
    n_tr = 4096
    log(f"[bench] generating {n_tr} traces")
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
    log(f"[bench] {n} events; first batched check")
    V.batch_check(ctx, traces)
    ctx.sync()
    viol = sum(t.violations().total for t in traces)
    ids = sum(sh.n_vars for sh in shapes)

    def step():
        V.batch_check(ctx, traces)

    def bytes_alg():
        return 4 * n + n + 4 * viol + ids

    def cpu_sample():
        v, k, m = _oracle_sample(inputs, 1 << 24)
        return v, f"oracle check of the first {k} traces ({m} events), one run"

    cfg = {"workload": "batched-4096-traces", "n_traces": n_tr, "n_events": n,
           "with_arrays": sum(1 for sh in shapes if sh.has_arrays), "violations": int(viol)}
    return dict(step=step, units=n, bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(traces, inputs),
                per_unit=lambda: bytes_alg() / n)


def wl_served(args, V, ctx, stream):
    """Served streams: 256 streams (trace lengths log-uniform in [2^16, 2^20], variables
    log-uniform in [8, 65,536], 20 % with array intervals), each submitting its trace in
    2^16-event chunks from host memory, all interleaved; the server admits, batches and
    checks them with the streams' status tables resident on the device.  A step opens
    the streams, submits every chunk, waits for every completion and closes the streams;
    it is timed on the host clock and includes the chunks' copies to the device."""
    from paper_1910_11110_amd import gen
    n_str, chunk = 256, 1 << 16
    log(f"[bench] generating {n_str} streams")
    shapes = gen.trace_shapes(n_str, args.seed, len_range=(1 << 16, 1 << 20))
    inputs = []
    for sh in shapes:
        ev, lo, hi = gen.trace_inputs(sh)
        inputs.append((ev, sh.n_vars, lo, hi))
    outs = [np.empty(ev.size, np.uint8) for ev, *_ in inputs]
    n = sum(ev.size for ev, *_ in inputs)
    srv = V.Server(ctx, 64 << 30)
    state = {"lat": [], "viol": 0}

    def step():
        sids = [srv.open(nv, lo, hi) for _ev, nv, lo, hi in inputs]
        maxc = max((ev.size + chunk - 1) // chunk for ev, *_ in inputs)
        want = 0
        for k in range(maxc):
            for i, (ev, *_r) in enumerate(inputs):
                a = k * chunk
                if a < ev.size:
                    srv.submit(sids[i], ev[a:a + chunk], outs[i][a:a + chunk])
                    want += 1
        lat, viol, got = [], 0, 0
        while got < want:
            cs = srv.poll()
            for c in cs:
                if c.status != 0:
                    raise RuntimeError(f"chunk {c.chunk} failed with {c.status}")
                lat.append(c.t_done - c.t_submit)
                viol += c.n_violations
            got += len(cs)
            if not cs:
                time.sleep(0.0002)
        for i, s_ in enumerate(sids):
            srv.close_stream(s_, inputs[i][1])
        state["lat"], state["viol"] = lat, viol

    def bytes_alg():
        return 4 * n + n + 4 * state["viol"] + sum(nv for _e, nv, *_r in inputs)

    def cpu_sample():
        v, k, m = _oracle_sample(inputs, 1 << 24)
        return v, f"oracle check of the first {k} streams' traces ({m} events), one run"

    def extra():
        lat = np.sort(np.asarray(state["lat"], np.float64)) * 1e3
        return {"serving": {"chunks_per_step": int(lat.size), "chunk_events": chunk,
                            "latency_ms_p50": round(float(lat[lat.size // 2]), 3),
                            "latency_ms_p99": round(float(lat[min(lat.size - 1, (lat.size * 99) // 100)]), 3),
                            "note": "submit-to-done per chunk; the step includes host-to-device copies"}}

    cfg = {"workload": "served-256-streams-2^16-chunks", "n_streams": n_str, "n_events": n}
    return dict(step=step, units=n, bytes_alg=bytes_alg, cpu=cpu_sample, config=cfg, keep=(srv, inputs, outs),
                per_unit=lambda: bytes_alg() / n, host_timed=True, extra=extra)


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
             "batched": wl_batched, "served": wl_served}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="components", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--comp-log2", type=int, default=23)
    ap.add_argument("--plain-log2", type=int, default=28)
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
    w = WORKLOADS[args.workload](args, V, ctx, stream)

    for _ in range(args.warmup):
        w["step"]()
    ctx.sync()
    torch.cuda.synchronize()
    # timed region: exactly `steps` steps, synchronized on both sides (a served step
    # waits for its own completions and runs on the server's streams: host clock)
    if w.get("host_timed"):
        a = time.perf_counter()
        for _ in range(args.steps):
            w["step"]()
        ctx.sync()
        ms_step = (time.perf_counter() - a) * 1e3 / args.steps
    else:
        with Timer(stream) as tm:
            for _ in range(args.steps):
                w["step"]()
        ctx.sync()
        ms_step = tm.ms / args.steps
    value = w["units"] / (ms_step / 1e3)

    # per-kernel durations: the same steps again with event pairs around each kernel
    ctx.profile(True)
    ctx.profile_reset()
    for _ in range(args.steps):
        w["step"]()
    prof = ctx.profile_read()
    ctx.profile(False)
    kernels = {k: {"ms_per_launch": ms / max(n, 1), "launches_per_step": n / args.steps, "ms_per_step": ms / args.steps}
               for k, (ms, n) in prof.items()}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"]) if kernels else None
    alg_step = w["bytes_alg"]()
    kb = w.get("kernel_bytes", {})
    # per kernel: its own algorithmic bytes per launch / its average launch time
    kroof = {}
    for k, (b, units, unit) in kb.items():
        if k in kernels and kernels[k]["ms_per_launch"] > 0:
            gbs = b / (kernels[k]["ms_per_launch"] / 1e3) / 1e9
            kroof[k] = {"bytes_per_launch": int(b), "units_per_launch": int(units), "unit": unit,
                        "achieved_GBs": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    roof = None
    if dom:
        d = kernels[dom]
        r = kroof.get(dom)
        achieved = r["achieved_GBs"] if r else None
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": r["frac"] if r else None, "traffic": traffic_for(dom, args.workload),
                "bytes_per_unit": round(r["bytes_per_launch"] / r["units_per_launch"], 3) if r else None,
                "units_per_launch": r["units_per_launch"] if r else None,
                "ms_per_launch": round(d["ms_per_launch"], 4)}
    pipeline = {"algorithmic_bytes_per_step": int(alg_step),
                "achieved_GBs": round(alg_step / (ms_step / 1e3) / 1e9, 2),
                "frac": round(alg_step / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        v, sample = w["cpu"]()
        cpu = {"value": round(v, 1), "unit": "events/s", "cores": 1, "kind": "oracle", "sample": sample}
    out = {
        "metric": "trace events checked/sec (bit-exact)",
        "value": round(value, 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": w["config"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "pipeline_roofline": pipeline,
        "kernel_rooflines": kroof,
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in kernels.items()},
        "source_digest": source_digest(),
    }
    if "extra" in w:
        out.update(w["extra"]())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
