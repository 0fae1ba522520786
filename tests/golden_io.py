"""Readers for the hand-written fixtures under tests/golden/."""
from __future__ import annotations

import os

import numpy as np

from paper_2109_09527_amd.synth import ADDV, REMV, HASV, ADDE, REME, HASE, make_ops

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_CODES = {"AV": ADDV, "RV": REMV, "HV": HASV, "AE": ADDE, "RE": REME, "HE": HASE}


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if line:
                yield line


def read_adt_scenario(name):
    """Returns (n, steps); a step is ("op", op_record, expected) or
    ("query", kind, src, expected_dist)."""
    n = None
    steps = []
    for line in _lines(name):
        lhs, _, rhs = line.partition("->")
        tok = lhs.split()
        if tok[0] == "n":
            n = int(tok[1])
        elif tok[0] == "query":
            steps.append(("query", tok[1], int(tok[2]), np.array(rhs.split(), dtype=np.int32)))
        else:
            code = _CODES[tok[0]]
            args = [int(x) for x in tok[1:]] + [0, 0, 0]
            u, v, w = args[0], args[1] if code >= ADDE else 0, args[2] if code == ADDE else 0
            op = make_ops(np.array([code]), np.array([u]), np.array([v]), np.array([w]))
            steps.append(("op", op, int(rhs)))
    return n, steps


def read_bc_fixture(name):
    d = {}
    for line in _lines(name):
        tok = line.split()
        d[tok[0]] = tok[1:]
    n = int(d["n"][0])
    arcs = np.array(d["arcs"], dtype=np.uint32).reshape(-1, 2)
    S = np.array(d["sources"], dtype=np.uint32)
    bc = np.array(d["bc"], dtype=np.float64)
    return n, arcs, S, bc
