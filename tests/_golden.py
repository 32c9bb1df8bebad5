"""Reader for the small text fixtures under tests/golden/ (comment lines start
with '#'; a bare word starts a named integer grid)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.strip() for ln in f if ln.strip() and not ln.lstrip().startswith("#")]


def read_grids(name):
    grids, cur = {}, None
    for ln in read_lines(name):
        toks = ln.split()
        if len(toks) == 1 and not toks[0].lstrip("-").isdigit():
            cur = toks[0]
            grids[cur] = []
        else:
            grids[cur].append([int(t) for t in toks])
    return {k: np.array(v, np.int64) for k, v in grids.items()}


def read_pairs(name):
    out = {}
    for ln in read_lines(name):
        k, v = ln.split()
        out[k] = int(v)
    return out
