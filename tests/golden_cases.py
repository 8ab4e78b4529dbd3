"""Reader of the hand-derived worked examples under tests/golden/ (format in
tests/golden/README.md): shared by the oracle's and the GPU path's checks."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MATRICES = ("left", "right", "image", "expect", "disp", "cost")


def _num(tok):
    return float(Fraction(tok))


def load_cases(name):
    """Cases of one fixture file: dicts of scalar fields (lists of numbers)
    and matrices (2-D float arrays)."""
    cases, cur, mat = [], None, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for raw in fh:
            line = raw.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "case":
                cur, mat = {"name": tok[1]}, None
            elif tok[0] == "end":
                cases.append({k: (np.array(v) if k in MATRICES else v) for k, v in cur.items()})
                cur, mat = None, None
            elif tok[0] in MATRICES and len(tok) == 1:
                mat = tok[0]
                cur[mat] = []
            elif mat is not None and not tok[0].isalpha():
                cur[mat].append([_num(t) for t in tok])
            else:
                mat = None
                cur[tok[0]] = tok[1] if tok[0] == "op" else [_num(t) for t in tok[1:]]
    assert cur is None, f"{name}: unterminated case"
    return cases


def ids(cases):
    return [c["name"] for c in cases]
