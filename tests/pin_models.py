"""Small independent models used to pin the oracle (tests only).

* ``halting_run``: the paper's small-step semantics taken literally -- a statement
  list is reduced until it is empty or stuck; no flag-and-skip continuation.
  Statuses are strings "V"/"I"; signatures are the printed strings, matched
  position by position.
* ``vectorpu_step``: the coherence-flag code of the VectorPU library as printed in
  the paper (Figure "Coherence control code"), acting on a (cpu, gpu) flag pair.
* ``ElementModel``: arrays whose every element carries its own status pair, for
  checking the overlapping-array theorem (Section 4) against the array-granular
  abstraction.
"""
from __future__ import annotations

import itertools

# printed signatures: input pattern -> output pattern, (local, remote)
SIGNATURES = {
    "Push": ("VX", "VV"),
    "Pull": ("XV", "VV"),
    "r": ("VX", "VX"),
    "w": ("XY", "VI"),
    "Noop": ("XY", "XY"),
}
OPS = ["r", "w", "Push", "Pull", "Noop"]


def _match(status: str, pattern: str):
    env = {}
    for s, p in zip(status, pattern):
        if p in "VI":
            if s != p:
                return None
        elif p in env and env[p] != s:
            return None
        else:
            env[p] = s
    return env


def _fire(status: str, op: str, remote: bool):
    """status is (local, remote) as a 2-char string; returns new status or None."""
    pin, pout = SIGNATURES[op]
    view = status[::-1] if remote else status
    env = _match(view, pin)
    if env is None:
        return None
    res = "".join(env.get(c, c) for c in pout)
    return res[::-1] if remote else res


def halting_run(program, store):
    """Reduce `program` (list of (op, remote, var)) from `store` (var -> 'VI' string)
    until it ends or is stuck.  Returns (list of statuses after each reduced step,
    index of the stuck statement or None)."""
    store = dict(store)
    posts = []
    for i, (op, remote, var) in enumerate(program):
        nxt = _fire(store[var], op, remote)
        if nxt is None:
            return posts, i
        store[var] = nxt
        posts.append(nxt)
    return posts, None


def code_of(s: str) -> int:
    return (1 if s[0] == "V" else 0) | (2 if s[1] == "V" else 0)


def str_of(code: int) -> str:
    return ("V" if code & 1 else "I") + ("V" if code & 2 else "I")


# -------------------------------------------------------------------------------------
# VectorPU coherence control code (host side = CPU, device side = GPU)
# -------------------------------------------------------------------------------------
def vectorpu_step(flags, mode: str, side: str):
    """flags = (cpu_coherent_unit, gpu_coherent_unit); mode in R/W/RW; side CPU/GPU."""
    cpu, gpu = flags
    if side == "CPU":
        if mode == "R":
            if not cpu:
                cpu = True  # download()
        elif mode == "W":
            cpu, gpu = True, False
        else:
            if not cpu:
                cpu = True  # download()
            gpu = False
    else:
        if mode == "R":
            if not gpu:
                gpu = True  # upload()
        elif mode == "W":
            gpu, cpu = True, False
        else:
            if not gpu:
                gpu = True  # upload()
            cpu = False
    return cpu, gpu


# -------------------------------------------------------------------------------------
# Element-level model of arrays
# -------------------------------------------------------------------------------------
def leq(a: str, b: str) -> bool:
    """Abstraction order: (V,I) <= (V,V), (I,V) <= (V,V), and reflexive."""
    return a == b or (b == "VV" and a in ("VI", "IV"))


class ElementModel:
    """Every address holds a status pair; every array has an abstract status pair.

    Declarations (mode, side, array) are translated as in Figure "Semantics of access
    modes and programs": the guarded transfer (Pull/Push on all elements of the array
    and on its abstract variable) and the write on the abstract variable.  Bodies
    access single elements.  Any stuck element step is recorded."""

    def __init__(self, n_addr: int, arrays: dict):
        self.elem = ["VI"] * n_addr
        self.arrays = dict(arrays)
        self.abs = {a: "VI" for a in arrays}
        self.stuck = []

    def _elem_step(self, addr, op, remote, tag):
        nxt = _fire(self.elem[addr], op, remote)
        if nxt is None:
            self.stuck.append(tag)
        else:
            self.elem[addr] = nxt

    def _abs_step(self, a, op, remote, tag):
        nxt = _fire(self.abs[a], op, remote)
        if nxt is None:
            self.stuck.append(tag)
        else:
            self.abs[a] = nxt

    def declare(self, mode: str, side: str, a: str):
        gpu = side == "GPU"
        lo, hi = self.arrays[a]
        if mode in ("R", "RW"):
            valid = self.abs[a][1] == "V" if gpu else self.abs[a][0] == "V"
            if not valid:
                t = "Push" if gpu else "Pull"
                for i in range(lo, hi):
                    self._elem_step(i, t, False, ("transfer", a, i))
                self._abs_step(a, t, False, ("transfer#", a))
        if mode in ("W", "RW"):
            self._abs_step(a, "w", gpu, ("w#", a))

    def access(self, op: str, side: str, a: str, i: int):
        lo, hi = self.arrays[a]
        assert lo <= i < hi
        self._elem_step(i, op, side == "GPU", (op, a, i))

    def abstraction_ok(self) -> bool:
        for a, (lo, hi) in self.arrays.items():
            for i in range(lo, hi):
                if not leq(self.abs[a], self.elem[i]):
                    return False
        return True


def all_programs(length: int, n_vars: int = 2):
    alphabet = [(op, remote, v) for v in range(n_vars) for op in OPS for remote in (False, True)]
    return itertools.product(alphabet, repeat=length)


# -------------------------------------------------------------------------------------
# structured programs, reduced literally
# -------------------------------------------------------------------------------------
def structured_run(stmts, store, choice: int, fuel: int):
    """The small-step rules of Figure "Operational semantics of validity status" on a
    statement list (tuples ("E", op, side, x), ("W", (kind, x), body), ("I", (kind, x),
    then, else); kind 0 isValid, 1 remIsValid, 2 the k-th choice is bit k of `choice`):
    the first statement of the configuration is reduced until the list is empty, a
    step is stuck, or `fuel` steps were taken.  Returns (steps, effects run, index of
    the stuck effect or None, completed, store)."""
    conf, store = list(stmts), dict(store)
    steps = effects = n_choice = 0
    while conf:
        if steps == fuel:
            return steps, effects, None, False, store
        st = conf.pop(0)
        if st[0] == "E":
            nxt = _fire(store[st[3]], OPS[st[1]], bool(st[2]))
            if nxt is None:
                return steps, effects, effects, False, store
            store[st[3]] = nxt
            steps += 1
            effects += 1
            continue
        kind, x = st[1]
        if kind == 0:
            c = store[x][0] == "V"       # rules valid / invalid
        elif kind == 1:
            c = store[x][1] == "V"       # rules rem-valid / rem-invalid
        else:
            c = bool((choice >> (n_choice % 64)) & 1)
            n_choice += 1
        steps += 1
        if st[0] == "W":                 # While-True / While-False
            conf = (list(st[2]) + [st] + conf) if c else conf
        else:                            # IF-True / IF-False
            conf = list(st[2] if c else st[3]) + conf
    return steps, effects, None, True, store
