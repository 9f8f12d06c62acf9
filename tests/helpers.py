"""Parsing of the golden fixtures (tests only)."""
from __future__ import annotations

import os

import numpy as np
import yaml

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
OPS = {"r": 0, "w": 1, "Push": 2, "Pull": 3, "Noop": 4}
MODES = {"R": 0, "W": 1, "RW": 2}
SIDES = {"CPU": 0, "GPU": 1}
PAIRS = {"(I,I)": 0, "(V,I)": 1, "(I,V)": 2, "(V,V)": 3}


def load_yaml(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return yaml.safe_load(f)


def ev(op, side, vid):
    return vid | (OPS[op] << 24) | (SIDES[side] << 27)


def decl(mode, side, vid):
    return vid | (MODES[mode] << 24) | (SIDES[side] << 27)


def parse_events(lines, ids):
    out = []
    for s in lines:
        op, side, var = s.split()
        out.append(ev(op, side, ids[var]))
    return np.array(out, dtype=np.uint32)


def effect_table():
    rows = []
    with open(os.path.join(GOLDEN, "effect_table.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            op, side, pre, post, stuck = line.split()
            rows.append((OPS[op], SIDES[side], PAIRS[pre], PAIRS[post], int(stuck)))
    return rows
