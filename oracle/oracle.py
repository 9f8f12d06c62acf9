"""Python access to the reference interpreter in ``vc_oracle.c``.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.  The library under test never loads it.

Every function here marshals numpy arrays into the C interpreter and back; no
arithmetic of the checked method is done in Python.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
STAMP = LIB + ".src"   # digest of the source the library was built from

_lib = None


def _digest() -> str:
    with open(SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _fresh() -> bool:
    if not (os.path.exists(LIB) and os.path.exists(STAMP)):
        return False
    with open(STAMP) as f:
        return f.read().strip() == _digest()


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation flags needed).  Called by
    the build entry point and by the test session's start-up, before any GPU work: a
    process that holds a GPU never starts a compiler."""
    if force or not _fresh():
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", tmp])
        os.replace(tmp, LIB)
        with open(STAMP, "w") as f:
            f.write(_digest() + "\n")
    return LIB


def load(path: str):
    """Load an oracle shared object and declare its signatures."""
    L = C.CDLL(path)
    P = C.c_void_p
    u64, u32, i32 = C.c_uint64, C.c_uint32, C.c_int
    pu64 = C.POINTER(C.c_uint64)
    L.oracle_check.argtypes = [P, u64, u32, P, P, P, P, u64, pu64, pu64, pu64]
    L.oracle_check.restype = i32
    L.oracle_check_count.argtypes = [P, u64, u32, P]
    L.oracle_check_count.restype = u64
    L.oracle_translate.argtypes = [P, u64, P, u32, P, P, P, u64, pu64, pu64]
    L.oracle_translate.restype = i32
    L.oracle_overlap_sets.argtypes = [P, P, u32, P, P, u64]
    L.oracle_overlap_sets.restype = u64
    L.oracle_check_overlap.argtypes = [P, u64, u32, P, P, P, P, P, P, u64, pu64, pu64, pu64, pu64, pu64]
    L.oracle_check_overlap.restype = i32
    L.oracle_check_dynamic.argtypes = [P, u64, u32, P, P, P, P, P, P, P, P, P, u64, pu64, pu64, pu64, pu64, pu64]
    L.oracle_check_dynamic.restype = i32
    L.oracle_check_spaces.argtypes = [P, u64, u32, u32, P, P, P, P, u64, pu64, pu64, pu64]
    L.oracle_check_spaces.restype = i32
    L.oracle_check_declared.argtypes = [P, u64, P, u32, P, P, P, P, P, P, P, i32, P, pu64]
    L.oracle_check_declared.restype = i32
    L.oracle_run_programs.argtypes = [P, u64, P, u32, P, P, u64, P, P, P, P, P, P, pu64]
    L.oracle_run_programs.restype = i32
    L.oracle_overlap_extend.argtypes = [P, i32, P, P, u32, P, i32]
    L.oracle_overlap_extend.restype = i32
    return L


def lib():
    """The built oracle.  It is never compiled here: a stale or missing library is an
    error (build it with build(), which the build entry point and the test session run)."""
    global _lib
    if _lib is None:
        if not _fresh():
            raise RuntimeError(f"{LIB} is missing or older than {SRC}; run oracle.oracle.build() first")
        _lib = load(LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(ValueError):
    pass


@dataclass
class CheckResult:
    status: np.ndarray      # uint8 per event: post | pre << 2 | stuck << 7
    final: np.ndarray       # uint8 per id
    violations: np.ndarray  # uint32 ascending event indices of stuck events
    first: int              # first stuck index, n if none
    n_induced: int = 0
    n_induced_stuck: int = 0


def check(events: np.ndarray, n_ids: int, init: np.ndarray | None = None) -> CheckResult:
    """Plain check: rules Effect / Remote Effect from the initial store."""
    ev = np.ascontiguousarray(events, dtype=np.uint32)
    n = ev.size
    ini = None if init is None else np.ascontiguousarray(init, dtype=np.uint8)
    st = np.empty(n, dtype=np.uint8)
    fin = np.empty(max(n_ids, 1), dtype=np.uint8)
    viol = np.empty(max(n, 1), dtype=np.uint32)
    nv, first, bad = C.c_uint64(), C.c_uint64(), C.c_uint64()
    rc = lib().oracle_check(_p(ev), n, n_ids, _p(ini), _p(st), _p(fin), _p(viol), viol.size,
                            C.byref(nv), C.byref(first), C.byref(bad))
    if rc == -1:
        raise OracleError(f"malformed event at index {bad.value}")
    if rc != 0:
        raise OracleError(f"oracle_check failed: {rc}")
    return CheckResult(st, fin[:n_ids], viol[:nv.value].copy(), first.value)


def check_count(events: np.ndarray, n_ids: int) -> int:
    ev = np.ascontiguousarray(events, dtype=np.uint32)
    return int(lib().oracle_check_count(_p(ev), ev.size, n_ids, None))


def translate(comp_off: np.ndarray, decls: np.ndarray, n_vars: int, body_off: np.ndarray | None = None,
              body: np.ndarray | None = None) -> np.ndarray:
    """Translated core trace of a component program (ids: real v, abstract n_vars + v)."""
    co = np.ascontiguousarray(comp_off, dtype=np.uint64)
    de = np.ascontiguousarray(decls, dtype=np.uint32)
    bo = None if body_off is None else np.ascontiguousarray(body_off, dtype=np.uint64)
    bd = None if body is None else np.ascontiguousarray(body, dtype=np.uint32)
    n_comp = co.size - 1
    nout, bad = C.c_uint64(), C.c_uint64()
    cap = int(de.size) * 5 + (0 if bd is None else int(bd.size))
    out = np.empty(max(cap, 1), dtype=np.uint32)
    rc = lib().oracle_translate(_p(co), n_comp, _p(de), n_vars, _p(bo), _p(bd), _p(out), out.size,
                                C.byref(nout), C.byref(bad))
    if rc == -1:
        raise OracleError(f"malformed declaration/body at index {bad.value}")
    if rc != 0:
        raise OracleError(f"oracle_translate failed: {rc}")
    return out[:nout.value].copy()


def overlap_sets(lo: np.ndarray, hi: np.ndarray):
    """CSR (off, nbr) of the overlap sets O(x) by the O(n^2) pair test."""
    lo = np.ascontiguousarray(lo, dtype=np.uint32)
    hi = np.ascontiguousarray(hi, dtype=np.uint32)
    n = lo.size
    off = np.empty(n + 1, dtype=np.uint64)
    # one pass when the neighbours fit a generous first guess, a second one otherwise
    nbr = np.empty(max(16 * n, 1), dtype=np.uint32)
    k = int(lib().oracle_overlap_sets(_p(lo), _p(hi), n, _p(off), _p(nbr), nbr.size))
    if k > nbr.size:
        nbr = np.empty(k, dtype=np.uint32)
        lib().oracle_overlap_sets(_p(lo), _p(hi), n, _p(off), _p(nbr), nbr.size)
    return off, nbr[:k].copy()


def check_overlap(events: np.ndarray, lo: np.ndarray, hi: np.ndarray, init: np.ndarray | None = None,
                  sets=None) -> CheckResult:
    """Check over arrays with the overlap rule for writes (induced RW on each
    overlapping array after the write)."""
    ev = np.ascontiguousarray(events, dtype=np.uint32)
    n_arrays = int(np.asarray(lo).size)
    off, nbr = overlap_sets(lo, hi) if sets is None else sets
    off = np.ascontiguousarray(off, dtype=np.uint64)
    nbr = np.ascontiguousarray(nbr if nbr.size else np.zeros(1, np.uint32), dtype=np.uint32)
    ini = None if init is None else np.ascontiguousarray(init, dtype=np.uint8)
    n = ev.size
    st = np.empty(n, dtype=np.uint8)
    fin = np.empty(max(n_arrays, 1), dtype=np.uint8)
    viol = np.empty(max(n, 1), dtype=np.uint32)
    nv, first, ni, nis, bad = (C.c_uint64() for _ in range(5))
    rc = lib().oracle_check_overlap(_p(ev), n, n_arrays, _p(off), _p(nbr), _p(ini), _p(st), _p(fin), _p(viol),
                                    viol.size, C.byref(nv), C.byref(first), C.byref(ni), C.byref(nis),
                                    C.byref(bad))
    if rc == -1:
        raise OracleError(f"malformed event at index {bad.value}")
    if rc != 0:
        raise OracleError(f"oracle_check_overlap failed: {rc}")
    return CheckResult(st, fin[:n_arrays], viol[:nv.value].copy(), first.value, ni.value, nis.value)


NO_MOTHER = 0xFFFFFFFF
OP_CREATE, OP_DESTROY = 6, 7


def check_dynamic(events: np.ndarray, lo: np.ndarray, hi: np.ndarray, mother: np.ndarray,
                  init: np.ndarray | None = None, sets=None) -> CheckResult:
    """Check with partial vectors created (op 6) and destroyed (op 7) during the trace:
    a created partial vector inherits its mother's status; a write induces RW on the
    arrays live at that point that overlap it (found in the list of live arrays, or,
    with sets = overlap_sets(lo, hi), among the overlapping arrays)."""
    ev = np.ascontiguousarray(events, dtype=np.uint32)
    lo = np.ascontiguousarray(lo, dtype=np.uint32)
    hi = np.ascontiguousarray(hi, dtype=np.uint32)
    mo = np.ascontiguousarray(mother, dtype=np.uint32)
    n_arrays = int(lo.size)
    ini = None if init is None else np.ascontiguousarray(init, dtype=np.uint8)
    n = ev.size
    st = np.empty(max(n, 1), dtype=np.uint8)
    fin = np.empty(max(n_arrays, 1), dtype=np.uint8)
    viol = np.empty(max(n, 1), dtype=np.uint32)
    nv, first, ni, nis, bad = (C.c_uint64() for _ in range(5))
    off = nbr = None
    if sets is not None:
        off = np.ascontiguousarray(sets[0], dtype=np.uint64)
        nbr = np.ascontiguousarray(sets[1] if sets[1].size else np.zeros(1, np.uint32), dtype=np.uint32)
    rc = lib().oracle_check_dynamic(_p(ev), n, n_arrays, _p(lo), _p(hi), _p(mo), _p(off), _p(nbr), _p(ini), _p(st),
                                    _p(fin),
                                    _p(viol), viol.size, C.byref(nv), C.byref(first), C.byref(ni), C.byref(nis),
                                    C.byref(bad))
    if rc == -1:
        raise OracleError(f"malformed event at index {bad.value}")
    if rc == -3:
        raise OracleError(f"array {bad.value} breaks the layout rules")
    if rc != 0:
        raise OracleError(f"oracle_check_dynamic failed: {rc}")
    return CheckResult(st[:n], fin[:n_arrays], viol[:nv.value].copy(), first.value, ni.value, nis.value)


def check_spaces(events: np.ndarray, n_ids: int, k: int, init: np.ndarray | None = None) -> CheckResult:
    """Check over k memory spaces: status is uint16 per event (post | pre << 4 |
    stuck << 15), final one k-bit code per id."""
    ev = np.ascontiguousarray(events, dtype=np.uint32)
    n = ev.size
    ini = None if init is None else np.ascontiguousarray(init, dtype=np.uint8)
    st = np.empty(max(n, 1), dtype=np.uint16)
    fin = np.empty(max(n_ids, 1), dtype=np.uint8)
    viol = np.empty(max(n, 1), dtype=np.uint32)
    nv, first, bad = C.c_uint64(), C.c_uint64(), C.c_uint64()
    rc = lib().oracle_check_spaces(_p(ev), n, n_ids, k, _p(ini), _p(st), _p(fin), _p(viol), viol.size,
                                   C.byref(nv), C.byref(first), C.byref(bad))
    if rc == -1:
        raise OracleError(f"malformed event at index {bad.value}")
    if rc != 0:
        raise OracleError(f"oracle_check_spaces failed: {rc}")
    return CheckResult(st[:n], fin[:n_ids], viol[:nv.value].copy(), first.value)


WD_TRANSFER, WD_READ, WD_WRITE, WD_UNWRITTEN, WD_OVERLAP, WD_ILL = 1, 2, 4, 8, 16, 128


def check_declared(comp_off, decls, n_vars: int, body_off, body, idx=None, lo=None, hi=None,
                   extend: bool = False, sets=None) -> np.ndarray:
    """Verdict byte per component of the well-declaredness conditions (bits WD_*);
    sets = overlap_sets(lo, hi) looks overlapping arrays up there (large inputs)."""
    co = np.ascontiguousarray(comp_off, dtype=np.uint64)
    de = np.ascontiguousarray(decls, dtype=np.uint32)
    bo = np.ascontiguousarray(body_off, dtype=np.uint64)
    bd = np.ascontiguousarray(body, dtype=np.uint32)
    ix = None if idx is None else np.ascontiguousarray(idx, dtype=np.uint32)
    l = None if lo is None else np.ascontiguousarray(lo, dtype=np.uint32)
    h = None if hi is None else np.ascontiguousarray(hi, dtype=np.uint32)
    n_comp = co.size - 1
    out = np.empty(max(n_comp, 1), np.uint8)
    bad = C.c_uint64()
    off = nbr = None
    if sets is not None:
        off = np.ascontiguousarray(sets[0], dtype=np.uint64)
        nbr = np.ascontiguousarray(sets[1] if sets[1].size else np.zeros(1, np.uint32), dtype=np.uint32)
    rc = lib().oracle_check_declared(_p(co), n_comp, _p(de), n_vars, _p(bo), _p(bd), _p(ix), _p(l), _p(h),
                                     _p(off), _p(nbr), 1 if extend else 0, _p(out), C.byref(bad))
    if rc == -1:
        raise OracleError(f"malformed declaration at index {bad.value}")
    if rc == -4:
        raise OracleError(f"malformed body word at index {bad.value}")
    if rc != 0:
        raise OracleError(f"oracle_check_declared failed: {rc}")
    return out[:n_comp]


@dataclass
class ProgramRuns:
    steps: np.ndarray    # reductions taken
    effects: np.ndarray  # effects run
    stuck: np.ndarray    # stuck effects
    first: np.ndarray    # effect index of the first stuck one (effects if none)
    done: np.ndarray     # 1 if the program completed within the fuel
    final: np.ndarray    # (n_prog, n_vars) final statuses


def run_programs(prog_off, words, n_vars: int, choice=None, init=None, fuel: int = 1 << 12) -> ProgramRuns:
    """Structured programs (While / If / sequence over effects), one per CSR range."""
    po = np.ascontiguousarray(prog_off, dtype=np.uint64)
    w = np.ascontiguousarray(words, dtype=np.uint32)
    ch = None if choice is None else np.ascontiguousarray(choice, dtype=np.uint64)
    ini = None if init is None else np.ascontiguousarray(init, dtype=np.uint8)
    n = po.size - 1
    out = [np.empty(max(n, 1), np.uint64) for _ in range(4)]
    done = np.empty(max(n, 1), np.uint8)
    fin = np.empty(max(n * n_vars, 1), np.uint8)
    bad = C.c_uint64()
    rc = lib().oracle_run_programs(_p(po), n, _p(w), n_vars, _p(ch), _p(ini), fuel, *[_p(o) for o in out], _p(done),
                                   _p(fin), C.byref(bad))
    if rc == -1:
        raise OracleError(f"malformed program word at index {bad.value}")
    if rc != 0:
        raise OracleError(f"oracle_run_programs failed: {rc}")
    return ProgramRuns(*[o[:n] for o in out], done[:n], fin[:n * n_vars].reshape(n, n_vars))


def overlap_extend(m: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """O(M): the declaration set M extended for overlapping arrays."""
    m = np.ascontiguousarray(m, dtype=np.uint32)
    lo = np.ascontiguousarray(lo, dtype=np.uint32)
    hi = np.ascontiguousarray(hi, dtype=np.uint32)
    cap = m.size + 2 * lo.size
    out = np.empty(max(cap, 1), dtype=np.uint32)
    k = lib().oracle_overlap_extend(_p(m), m.size, _p(lo), _p(hi), lo.size, _p(out), out.size)
    if k < 0:
        raise OracleError("overlap_extend capacity")
    return out[:k].copy()


# status byte fields
def post(st):
    return np.asarray(st) & 3


def pre(st):
    return (np.asarray(st) >> 2) & 3


def stuck(st):
    return (np.asarray(st) >> 7) & 1
