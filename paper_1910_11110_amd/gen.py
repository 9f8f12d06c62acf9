"""Seeded synthetic inputs for the validity-status checker.

This module draws the *inputs* of the workloads (event traces, access-mode
declarations, array intervals, trace shapes, arrival times).  It contains none of
the checked method's arithmetic: no status, no effect, no transfer decision.  Both
the CPU oracle and the HIP path consume what it produces, and neither imports the
other.

Random numbers come from a counter-based SplitMix64 (G. Steele, D. Lea, C. Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014).  Draw ``i`` of
stream ``(seed, stream)`` is ``mix64(base + (i + 1) * GAMMA)`` where
``base = mix64(mix64(seed) ^ (stream * GAMMA))``.  Every field of every workload
uses its own stream, so any slice of a workload can be regenerated without the
rest.

Wire formats produced here (they are the library's input formats):

* event   : bits 0-23 variable id, bits 24-26 op (0 r, 1 w, 2 Push, 3 Pull,
            4 Noop), bit 27 side (0 = CPU / local, 1 = GPU / remote), bits 28-31 zero.
* decl    : bits 0-23 variable, bits 24-25 mode (0 R, 1 W, 2 RW), bit 27 side.
* comp_off: uint64 CSR offsets of each component's declarations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream identifiers (one per drawn field)
S_VAR, S_OP, S_SIDE = 1, 2, 3
S_K, S_ZIPF, S_MODE, S_CSIDE = 10, 11, 12, 13
S_LEN, S_LO, S_ARR = 20, 21, 22
S_TLEN, S_TVARS, S_TARR, S_TSEED = 30, 31, 32, 33
S_ARRIVE = 40
S_DMOTHER, S_DLEN, S_DLO, S_DLIFE, S_DCPOS, S_DDPOS, S_DVAR = 50, 51, 52, 53, 54, 55, 56
S_KVAR, S_KOP, S_KA, S_KB = 60, 61, 62, 63
S_WK, S_WVAR, S_WMODE, S_WSIDE, S_WEL, S_WERR, S_WERRK = 70, 71, 72, 73, 74, 75, 76
S_PT, S_PPICK, S_PCHOICE, S_PINIT = 80, 81, 82, 83

OP_R, OP_W, OP_PUSH, OP_PULL, OP_NOOP = 0, 1, 2, 3, 4
MODE_R, MODE_W, MODE_RW = 0, 1, 2
CPU, GPU = 0, 1


def _mix64_inplace(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser, in place on a uint64 array."""
    t = np.empty_like(z)
    with np.errstate(over="ignore"):
        np.right_shift(z, np.uint64(30), out=t)
        z ^= t
        z *= _M1
        np.right_shift(z, np.uint64(27), out=t)
        z ^= t
        z *= _M2
        np.right_shift(z, np.uint64(31), out=t)
        z ^= t
    return z


def _mix64(z: np.ndarray) -> np.ndarray:
    return _mix64_inplace(np.array(z, dtype=np.uint64, copy=True))


_POOL = None
_CHUNK = 1 << 22


def _pool():
    global _POOL
    if _POOL is None:
        import concurrent.futures as cf
        import os
        _POOL = cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1))
    return _POOL


def _chunked(n: int, fn, out: np.ndarray) -> np.ndarray:
    """Fills out[a:b] = fn(a, b) over chunks, in parallel (numpy releases the GIL)."""
    if n <= _CHUNK:
        if n:
            out[:n] = fn(0, n)
        return out
    spans = [(a, min(n, a + _CHUNK)) for a in range(0, n, _CHUNK)]

    def run(ab):
        a, b = ab
        out[a:b] = fn(a, b)

    list(_pool().map(run, spans))
    return out


def _stream_base(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = _mix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))
        t = np.array([stream & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64) * GAMMA
        return _mix64(s ^ t)[0]


def draws(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """``count`` 64-bit draws of stream (seed, stream), starting at draw ``start``."""
    base = _stream_base(seed, stream)

    def fn(a, b):
        z = np.arange(start + a + 1, start + b + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z *= GAMMA
            z += base
        return _mix64_inplace(z)

    return _chunked(count, fn, np.empty(count, dtype=np.uint64))


def draws_at(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Draws of stream (seed, stream) at the given counter indices."""
    base = _stream_base(seed, stream)
    with np.errstate(over="ignore"):
        return _mix64(base + (np.asarray(idx, dtype=np.uint64) + np.uint64(1)) * GAMMA)


def below(u: np.ndarray, n: int) -> np.ndarray:
    """Map 64-bit draws to integers in [0, n) by multiply-shift of the top 32 bits."""
    assert 0 < n <= (1 << 32)
    hi = (u >> np.uint64(32)).astype(np.uint64)
    with np.errstate(over="ignore"):
        return ((hi * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


def unit(u: np.ndarray) -> np.ndarray:
    """Map 64-bit draws to floats in [0, 1) with 53 random bits."""
    return (u >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def pack_events(var, op, side) -> np.ndarray:
    var = np.asarray(var, dtype=np.uint32)
    op = np.asarray(op, dtype=np.uint32)
    side = np.asarray(side, dtype=np.uint32)
    return (var | (op << np.uint32(24)) | (side << np.uint32(27))).astype(np.uint32)


def pack_decls(var, mode, side) -> np.ndarray:
    var = np.asarray(var, dtype=np.uint32)
    mode = np.asarray(mode, dtype=np.uint32)
    side = np.asarray(side, dtype=np.uint32)
    return (var | (mode << np.uint32(24)) | (side << np.uint32(27))).astype(np.uint32)


# --------------------------------------------------------------------------------------
# plain traces: uniform variable, uniform op over the five effects, fair side
# --------------------------------------------------------------------------------------
def plain_events(n: int, n_ids: int, seed: int, start: int = 0, chunk: int = 1 << 24) -> np.ndarray:
    """Events ``start .. start+n`` of the plain-trace law (variable uniform in
    [0, n_ids), op uniform over r/w/Push/Pull/Noop, side CPU/GPU with p = 0.5)."""
    out = np.empty(n, dtype=np.uint32)
    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        var = below(draws(seed, S_VAR, start + a, m), n_ids)
        op = below(draws(seed, S_OP, start + a, m), 5)
        side = draws(seed, S_SIDE, start + a, m) >> np.uint64(63)
        out[a:a + m] = pack_events(var, op, side)
    return out


# --------------------------------------------------------------------------------------
# component traces: declarations of VectorPU-style components
# --------------------------------------------------------------------------------------
_zipf_cache: dict = {}


def zipf_cdf(n_vars: int, s: float) -> np.ndarray:
    """Cumulative distribution of P(k) proportional to (k+1)^-s over k in [0, n_vars)."""
    key = (n_vars, s)
    if key not in _zipf_cache:
        w = np.power(np.arange(1, n_vars + 1, dtype=np.float64), -s)
        c = np.cumsum(w)
        c /= c[-1]
        c[-1] = 1.0
        guide_n = 1 << 22
        guide = np.searchsorted(c, np.arange(guide_n, dtype=np.float64) / guide_n, side="right")
        _zipf_cache[key] = (c, guide)
    return _zipf_cache[key][0]


def zipf_inverse(u: np.ndarray, n_vars: int, s: float) -> np.ndarray:
    """Inverse CDF: the smallest k with cdf[k] > u (searchsorted side='right'), found
    from a guide table and a short forward walk; identical to a binary search."""
    zipf_cdf(n_vars, s)
    c, guide = _zipf_cache[(n_vars, s)]
    gn = guide.size

    def fn(a, b):
        uu = u[a:b]
        k = guide[np.minimum((uu * gn).astype(np.int64), gn - 1)]
        while True:
            k_ok = np.minimum(k, n_vars - 1)
            step = (c[k_ok] <= uu) & (k < n_vars - 1)
            if not step.any():
                break
            k = k + step
        return np.minimum(k, n_vars - 1)

    return _chunked(u.size, fn, np.empty(u.size, dtype=np.int64))


@dataclass
class ComponentTrace:
    n_vars: int
    comp_off: np.ndarray  # uint64, n_comp + 1
    decls: np.ndarray     # uint32

    @property
    def n_comp(self) -> int:
        return len(self.comp_off) - 1


def component_trace(n_comp: int, n_vars: int, seed: int, kmax: int = 8, zipf_s: float = 1.1,
                     p_modes=(0.5, 0.3, 0.2)) -> ComponentTrace:
    """``n_comp`` components; each declares k ~ U{1..kmax} distinct variables drawn by
    Zipf(zipf_s) over [0, n_vars) (a repeated draw is redrawn until distinct); each
    declaration gets mode R/W/RW with probabilities ``p_modes``; each component is
    placed on CPU or GPU with p = 0.5."""
    assert kmax <= n_vars
    k = below(draws(seed, S_K, 0, n_comp), kmax) + 1
    # column j holds the j-th declared variable of every component
    cols = zipf_inverse(unit(draws(seed, S_ZIPF, 0, n_comp * kmax)), n_vars, zipf_s).reshape(n_comp, kmax).T.copy()
    attempt = 1
    for j in range(1, kmax):
        # rows whose j-th draw repeats an earlier one are redrawn until distinct
        rows = np.nonzero(k > j)[0]
        while rows.size:
            cj = cols[j, rows]
            dup = np.zeros(rows.size, dtype=bool)
            for i in range(j):
                dup |= cj == cols[i, rows]
            rows = rows[dup]
            if rows.size == 0:
                break
            u = unit(draws_at(seed, S_ZIPF + 1000 * attempt, rows.astype(np.uint64) * np.uint64(kmax) + np.uint64(j)))
            cols[j, rows] = zipf_inverse(u, n_vars, zipf_s)
            attempt += 1
    ids = cols.T
    mask = np.arange(kmax)[None, :] < k[:, None]
    var = ids[mask]
    n_decl = var.size
    mu = unit(draws(seed, S_MODE, 0, n_decl))
    mode = np.where(mu < p_modes[0], MODE_R, np.where(mu < p_modes[0] + p_modes[1], MODE_W, MODE_RW))
    cside = (draws(seed, S_CSIDE, 0, n_comp) >> np.uint64(63)).astype(np.int64)
    side = np.repeat(cside, k)
    comp_off = np.zeros(n_comp + 1, dtype=np.uint64)
    np.cumsum(k, out=comp_off[1:])
    return ComponentTrace(n_vars, comp_off, pack_decls(var, mode, side))


# --------------------------------------------------------------------------------------
# overlapping arrays
# --------------------------------------------------------------------------------------
def intervals(n_arrays: int, seed: int, space: int = 1 << 24, max_len: int = 4096):
    """Half-open intervals [lo, hi): length log-uniform integer in [1, max_len]
    (floor of exp(u ln(max_len + 1))), then lo uniform in [0, space - len]."""
    u = unit(draws(seed, S_LEN, 0, n_arrays))
    ln = np.floor(np.exp(u * math.log(max_len + 1))).astype(np.int64)
    ln = np.clip(ln, 1, max_len)
    lo = np.empty(n_arrays, dtype=np.int64)
    ulo = draws(seed, S_LO, 0, n_arrays)
    # per-element bound space - len + 1
    hi32 = (ulo >> np.uint64(32)).astype(np.uint64)
    bound = (space - ln + 1).astype(np.uint64)
    with np.errstate(over="ignore"):
        lo[:] = ((hi32 * bound) >> np.uint64(32)).astype(np.int64)
    return lo.astype(np.uint32), (lo + ln).astype(np.uint32)


# --------------------------------------------------------------------------------------
# component programs with explicit bodies (for the well-declaredness check)
# --------------------------------------------------------------------------------------
@dataclass
class DeclaredProgram:
    comp_off: np.ndarray
    decls: np.ndarray
    n_vars: int
    body_off: np.ndarray
    body: np.ndarray
    idx: np.ndarray | None   # element index per body event (arrays), else None
    lo: np.ndarray | None
    hi: np.ndarray | None


def declared_program(n_comp: int, n_vars: int, seed: int, arrays: bool = True, space: int = 1 << 24,
                     max_len: int = 64, kmax: int = 4, p_err: float = 0.05) -> DeclaredProgram:
    """Components declaring k ~ U{1..kmax} distinct variables (uniform ids, redrawn until
    distinct), modes R/W/RW with p 0.5/0.3/0.2, one side per component (p = 0.5).  The body
    visits every element of every declared variable in declaration order: R reads it with
    p = 0.5, W writes it, RW reads it with p = 0.5 and writes it with p = 0.5 (a read before
    the write).  With arrays, variables are intervals (lengths log-uniform in [1, max_len])
    and body events carry element indices; without, every variable has one element.  A
    fraction p_err of components has its first body event altered: its side flipped, or
    (one in three) turned into a Push."""
    k = below(draws(seed, S_WK, 0, n_comp), kmax) + 1
    cols = below(draws(seed, S_WVAR, 0, n_comp * kmax), n_vars).reshape(n_comp, kmax).T.copy()
    attempt = 1
    for j in range(1, kmax):
        rows = np.nonzero(k > j)[0]
        while rows.size:
            cj = cols[j, rows]
            dup = np.zeros(rows.size, dtype=bool)
            for i in range(j):
                dup |= cj == cols[i, rows]
            rows = rows[dup]
            if rows.size == 0:
                break
            cols[j, rows] = below(draws_at(seed, S_WVAR + 1000 * attempt,
                                           rows.astype(np.uint64) * np.uint64(kmax) + np.uint64(j)), n_vars)
            attempt += 1
    mask = np.arange(kmax)[None, :] < k[:, None]
    var = cols.T[mask].astype(np.int64)
    n_decl = var.size
    mu = unit(draws(seed, S_WMODE, 0, n_decl))
    mode = np.where(mu < 0.5, MODE_R, np.where(mu < 0.8, MODE_W, MODE_RW))
    cside = (draws(seed, S_WSIDE, 0, n_comp) >> np.uint64(63)).astype(np.int64)
    side = np.repeat(cside, k)
    comp_off = np.zeros(n_comp + 1, dtype=np.uint64)
    np.cumsum(k, out=comp_off[1:])
    if arrays:
        lo, hi = intervals(n_vars, seed, space, max_len)
        ln = (hi.astype(np.int64) - lo.astype(np.int64))[var]
    else:
        lo = hi = None
        ln = np.ones(n_decl, np.int64)
    # one entry per (declaration, element), in declaration order
    de = np.repeat(np.arange(n_decl), ln)
    start = np.cumsum(ln) - ln
    el = np.arange(de.size) - np.repeat(start, ln)
    u = unit(draws(seed, S_WEL, 0, 2 * de.size)).reshape(2, de.size)
    m = mode[de]
    rd = ((m == MODE_R) & (u[0] < 0.5)) | ((m == MODE_RW) & (u[0] < 0.5))
    wr = (m == MODE_W) | ((m == MODE_RW) & (u[1] < 0.5))
    # each entry gives a read then a write
    cnt = rd.astype(np.int64) + wr.astype(np.int64)
    ent = np.repeat(np.arange(de.size), cnt)
    first_of = np.cumsum(cnt) - cnt
    is_second = (np.arange(ent.size) - first_of[ent]) == 1
    op = np.where(rd[ent] & ~is_second, OP_R, OP_W)
    bd = de[ent]
    body = pack_events(var[bd], op, side[bd])
    idx = el[ent].astype(np.uint32)
    comp_of_decl = np.repeat(np.arange(n_comp), k)
    body_cnt = np.bincount(comp_of_decl[bd], minlength=n_comp)
    body_off = np.zeros(n_comp + 1, dtype=np.uint64)
    np.cumsum(body_cnt, out=body_off[1:])
    # faults: the first body event of a few components
    ue = unit(draws(seed, S_WERR, 0, n_comp))
    uk = below(draws(seed, S_WERRK, 0, n_comp), 3)
    bad = np.nonzero((ue < p_err) & (body_cnt > 0))[0]
    fpos = body_off[bad].astype(np.int64)
    push = uk[bad] == 0
    w = body[fpos]
    body[fpos] = np.where(push, (w & np.uint32(0x08FFFFFF)) | np.uint32(OP_PUSH << 24), w ^ np.uint32(1 << 27))
    decls = pack_decls(var, mode, side)
    return DeclaredProgram(comp_off, decls, n_vars, body_off, body, idx if arrays else None, lo, hi)


# --------------------------------------------------------------------------------------
# structured programs (While / If / sequences of effects)
# --------------------------------------------------------------------------------------
K_VALID, K_REMVALID, K_CHOICE = 0, 1, 2


def program_words(stmts) -> list:
    """Prefix serialisation of a statement list: an effect is its event word; While is
    (1 << 30 | kind << 24 | x, body length) then the body; If is (2 << 30 | kind << 24 |
    x, then length, else length) then both branches.  Statements are tuples ("E", op,
    side, x), ("W", (kind, x), body), ("I", (kind, x), then, else)."""
    out = []
    for st in stmts:
        if st[0] == "E":
            out.append(int(st[3]) | (int(st[1]) << 24) | (int(st[2]) << 27))
        elif st[0] == "W":
            body = program_words(st[2])
            out += [(1 << 30) | (st[1][0] << 24) | st[1][1], len(body)] + body
        else:
            a, b = program_words(st[2]), program_words(st[3])
            out += [(2 << 30) | (st[1][0] << 24) | st[1][1], len(a), len(b)] + a + b
    return out


def random_program(rng: np.random.Generator, n_vars: int, max_words: int, depth: int = 0) -> list:
    """A random statement list of at most about max_words words: effects (op uniform,
    side and variable uniform), While and If on isValid / remIsValid / choice
    conditions, nested up to depth 3."""
    out, used = [], 0
    while used < max_words:
        u = rng.random()
        if depth < 3 and u < 0.12 and max_words - used > 6:
            cond = (int(rng.choice(3, p=[0.4, 0.4, 0.2])), int(rng.integers(n_vars)))
            body = random_program(rng, n_vars, int(rng.integers(1, max(2, (max_words - used) // 3))), depth + 1)
            out.append(("W", cond, body))
        elif depth < 3 and u < 0.3 and max_words - used > 8:
            cond = (int(rng.choice(3, p=[0.4, 0.4, 0.2])), int(rng.integers(n_vars)))
            k = max(2, (max_words - used) // 4)
            out.append(("I", cond, random_program(rng, n_vars, int(rng.integers(0, k)), depth + 1),
                        random_program(rng, n_vars, int(rng.integers(0, k)), depth + 1)))
        else:
            out.append(("E", int(rng.integers(5)), int(rng.integers(2)), int(rng.integers(n_vars))))
        used = len(program_words(out))
    return out


@dataclass
class Programs:
    prog_off: np.ndarray
    words: np.ndarray
    n_vars: int
    choice: np.ndarray   # uint64 per program: outcomes of its choice conditions
    init: np.ndarray     # (n_prog * n_vars) initial statuses


def structured_programs(n_prog: int, n_vars: int, seed: int, n_templates: int = 4096,
                        max_words: int = 64) -> Programs:
    """n_prog programs over n_vars variables each, drawn uniformly from n_templates
    random templates, each with its own choice word and initial statuses drawn
    uniformly from (V,I), (I,V), (V,V)."""
    rng = np.random.default_rng(seed)
    temps = [np.array(program_words(random_program(rng, n_vars, max_words)), np.uint32) for _ in range(n_templates)]
    pick = below(draws(seed, S_PPICK, 0, n_prog), n_templates)
    lens = np.array([t.size for t in temps], np.int64)[pick]
    prog_off = np.zeros(n_prog + 1, np.uint64)
    np.cumsum(lens, out=prog_off[1:])
    flat = np.concatenate(temps)
    toff = np.zeros(n_templates + 1, np.int64)
    np.cumsum([t.size for t in temps], out=toff[1:])
    src = np.repeat(toff[pick], lens) + (np.arange(int(lens.sum())) - np.repeat(prog_off[:-1].astype(np.int64), lens))
    words = flat[src]
    choice = draws(seed, S_PCHOICE, 0, n_prog)
    init = (below(draws(seed, S_PINIT, 0, n_prog * n_vars), 3) + 1).astype(np.uint8)
    return Programs(prog_off, words, n_vars, choice, init)


# --------------------------------------------------------------------------------------
# k memory spaces
# --------------------------------------------------------------------------------------
def space_events(n: int, n_ids: int, k: int, seed: int) -> np.ndarray:
    """k-space event words: variable uniform in [0, n_ids), op uniform over {r, w, copy,
    Noop}, location a uniform in [0, k) (0 for Noop), copy target b uniform in [0, k)."""
    x = below(draws(seed, S_KVAR, 0, n), n_ids).astype(np.uint32)
    op = below(draws(seed, S_KOP, 0, n), 4).astype(np.uint32)
    a = below(draws(seed, S_KA, 0, n), k).astype(np.uint32)
    b = below(draws(seed, S_KB, 0, n), k).astype(np.uint32)
    a = np.where(op == 3, np.uint32(0), a)
    b = np.where(op == 2, b, np.uint32(0))
    return x | (op << np.uint32(24)) | (a << np.uint32(26)) | (b << np.uint32(28))


# --------------------------------------------------------------------------------------
# partial vectors created and destroyed during a trace
# --------------------------------------------------------------------------------------
NO_MOTHER = 0xFFFFFFFF
OP_CREATE, OP_DESTROY = 6, 7


@dataclass
class DynamicTrace:
    events: np.ndarray  # uint32 event words (ops 0-4, 6 create, 7 destroy)
    lo: np.ndarray
    hi: np.ndarray
    mother: np.ndarray  # uint32, NO_MOTHER for a vector


def dynamic_trace(n: int, n_vectors: int, n_pvectors: int, seed: int, space: int = 1 << 24,
                  max_len: int = 4096, p_initial: float = 0.25, p_destroyed: float = 0.5) -> DynamicTrace:
    """Vectors tile the address space (vector v holds [v L, (v + 1) L), L = space /
    n_vectors) and live for the whole trace.  Each partial vector has a mother drawn
    uniformly, a length log-uniform in [1, min(max_len, L)] and a start uniform inside
    its mother.  A fraction ``p_initial`` of partial vectors is live from the start; the
    others are created at a uniform position; a fraction ``p_destroyed`` of all partial
    vectors is destroyed at a uniform later position.  Events draw the array uniformly
    over all ids, op and side as in the plain law; an event whose array is not live at
    its position goes to the array's mother instead; create and destroy words replace
    the events at their positions (positions drawn distinct)."""
    L = space // n_vectors
    n_ids = n_vectors + n_pvectors
    lo = np.empty(n_ids, np.int64)
    hi = np.empty(n_ids, np.int64)
    mother = np.full(n_ids, NO_MOTHER, np.uint32)
    lo[:n_vectors] = np.arange(n_vectors, dtype=np.int64) * L
    hi[:n_vectors] = lo[:n_vectors] + L
    m = below(draws(seed, S_DMOTHER, 0, n_pvectors), n_vectors).astype(np.int64)
    cap = min(max_len, L)
    u = unit(draws(seed, S_DLEN, 0, n_pvectors))
    ln = np.clip(np.floor(np.exp(u * math.log(cap + 1))).astype(np.int64), 1, cap)
    off = (unit(draws(seed, S_DLO, 0, n_pvectors)) * (L - ln + 1)).astype(np.int64)
    off = np.minimum(off, L - ln)
    lo[n_vectors:] = lo[m] + off
    hi[n_vectors:] = lo[n_vectors:] + ln
    mother[n_vectors:] = m.astype(np.uint32)
    # lifetimes: create / destroy positions, all distinct
    ul = unit(draws(seed, S_DLIFE, 0, 2 * n_pvectors)).reshape(2, n_pvectors)
    created = ul[0] >= p_initial
    destroyed = ul[1] < p_destroyed
    k = int(created.sum() + destroyed.sum())
    assert k <= n, "more lifetime events than positions"
    # distinct positions: a random subset of size k in increasing order, dealt out in a
    # seeded order
    pool = np.unique(below(draws(seed, S_DCPOS, 0, 4 * k + 16), n))
    while pool.size < k:
        pool = np.unique(np.concatenate([pool, below(draws(seed, S_DDPOS, pool.size, 4 * k + 16), n)]))
    order = np.argsort(draws(seed, S_DDPOS, 1 << 40, pool.size))
    pos = pool[order][:k]
    ids = np.nonzero(created)[0]
    cpos = np.full(n_pvectors, -1, np.int64)
    cpos[ids] = pos[:ids.size]
    dids = np.nonzero(destroyed)[0]
    dcand = pos[ids.size:ids.size + dids.size]
    dpos = np.full(n_pvectors, n + 1, np.int64)
    # a destroy goes after the create: swap the two positions when drawn the other way
    c_of_d = cpos[dids]
    swap = c_of_d > dcand
    dpos[dids] = np.where(swap, c_of_d, dcand)
    cpos[dids[swap]] = dcand[swap]
    ev = plain_events(n, n_ids, seed)
    x = (ev & np.uint32(0xFFFFFF)).astype(np.int64)
    t = np.arange(n, dtype=np.int64)
    pv = x >= n_vectors
    j = np.where(pv, x - n_vectors, 0)
    dead = pv & ((cpos[j] >= t) | (dpos[j] <= t))
    x = np.where(dead, mother[np.where(pv, x, 0)].astype(np.int64), x)
    ev = (ev & np.uint32(0xFF000000)) | x.astype(np.uint32)
    cw = np.nonzero(cpos >= 0)[0]
    ev[cpos[cw]] = (n_vectors + cw).astype(np.uint32) | np.uint32(OP_CREATE << 24)
    dw = np.nonzero(dpos <= n)[0]
    ev[dpos[dw]] = (n_vectors + dw).astype(np.uint32) | np.uint32(OP_DESTROY << 24)
    return DynamicTrace(ev, lo.astype(np.uint32), hi.astype(np.uint32), mother)


# --------------------------------------------------------------------------------------
# batched / served trace shapes
# --------------------------------------------------------------------------------------
@dataclass
class TraceShape:
    length: int
    n_vars: int
    has_arrays: bool
    seed: int


def _log_uniform_int(u: np.ndarray, lo: int, hi: int) -> np.ndarray:
    v = np.floor(np.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo)))).astype(np.int64)
    return np.clip(v, lo, hi)


def trace_shapes(n_traces: int, seed: int, len_range=(100, 1_000_000), vars_range=(8, 65536),
                 p_arrays: float = 0.2, start: int = 0) -> list:
    """Shapes of independent traces: length and variable count log-uniform integers in
    the given ranges, a fraction ``p_arrays`` of traces carrying array intervals."""
    lens = _log_uniform_int(unit(draws(seed, S_TLEN, start, n_traces)), *len_range)
    nv = _log_uniform_int(unit(draws(seed, S_TVARS, start, n_traces)), *vars_range)
    arr = unit(draws(seed, S_TARR, start, n_traces)) < p_arrays
    tseed = draws(seed, S_TSEED, start, n_traces)
    return [TraceShape(int(lens[i]), int(nv[i]), bool(arr[i]), int(tseed[i] & np.uint64(0x7FFFFFFFFFFFFFFF)))
            for i in range(n_traces)]


def trace_inputs(shape: TraceShape):
    """Events (and intervals if the trace carries arrays) of one trace shape."""
    ev = plain_events(shape.length, shape.n_vars, shape.seed)
    if shape.has_arrays:
        lo, hi = intervals(shape.n_vars, shape.seed)
        return ev, lo, hi
    return ev, None, None


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate over [0, duration)."""
    n_est = int(rate * duration * 1.5 + 64)
    u = unit(draws(seed, S_ARRIVE, 0, n_est))
    gaps = -np.log1p(-u) / rate
    t = np.cumsum(gaps)
    return t[t < duration]


# --------------------------------------------------------------------------------------
# workload presets (sizes of the workloads the checker is measured on)
# --------------------------------------------------------------------------------------
PLAIN_SMALL = dict(n=10_000, n_ids=64)              # single trace, 64 scalar variables
PLAIN_LARGE = dict(n=1 << 28, n_ids=64)             # same law at 2^28 events (1 GiB)
COMPONENTS = dict(n_comp=1 << 23, n_vars=1 << 20)   # VectorPU-style component trace
OVERLAP = dict(n_arrays=1 << 16, n_events=1 << 24)  # overlapping arrays
BATCH = dict(n_traces=4096)                         # batched traces
SERVE = dict(rate=2000.0, duration=60.0, chunk=1 << 16, budget=64 << 30)
