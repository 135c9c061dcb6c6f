"""Reading the stored oracle results (c4_expected.txt, c5_pool_expected.txt)
that make_expected.py writes.  Holds no arithmetic of the method and imports
neither the oracle nor the device library, so any reader may use it.

File format (text, one request per line, in the workload's request order):
    fingerprint <sha256 of the workload definition>
    sel  <i> <sampled_rows> <kept_blocks> <count_0> ... <count_{m-1}>
    join <j> <join_card> <ndv_R> <ndv_S> <n_R> <n_S> <f1_R> <f1_S> <f2_R> <f2_S>
"""
from __future__ import annotations

import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
FILES = {"c4": os.path.join(HERE, "c4_expected.txt"), "c5": os.path.join(HERE, "c5_pool_expected.txt")}
JOIN_FIELDS = ["join_card", "ndv_R", "ndv_S", "n_R", "n_S", "f1_R", "f1_S", "f2_R", "f2_S"]


def _col(c):
    return [c.dtype, c.kind, c.seed, c.table, c.col, c.lo, c.span, repr(c.zipf_s), c.zipf_n,
            c.noise_lo, c.noise_span, c.base_col]


def _table(t):
    return [t.n_rows, t.table_id, [_col(c) for c in t.cols]]


def _spec(s):
    return [s.seed, repr(float(s.rate)), s.block_rows]


def fingerprint(w) -> str:
    """sha256 of a canonical dump of everything that decides the results."""
    doc = {
        "tables": [_table(t) for t in w.tables],
        "sel": [[r.table, [[[c, op, [repr(v) for v in vals]] for (c, op, vals) in p] for p in r.preds],
                 _spec(r.spec)] for r in w.sel],
        "joins": [[_table(j.r), _table(j.s), _spec(j.spec_r), _spec(j.spec_s)] for j in w.joins],
        "order": [list(o) for o in w.order],
    }
    return hashlib.sha256(json.dumps(doc, sort_keys=True).encode()).hexdigest()


def load(name: str, w=None):
    """-> {("sel", i): (counts list, sampled, kept), ("join", j): dict}; checks the fingerprint
    when a workload is given."""
    out = {}
    with open(FILES[name]) as f:
        head = f.readline().split()
        assert head[0] == "fingerprint"
        if w is not None and head[1] != fingerprint(w):
            raise ValueError("%s was written for another workload definition" % FILES[name])
        for line in f:
            p = line.split()
            if p[0] == "sel":
                out[("sel", int(p[1]))] = ([int(x) for x in p[4:]], int(p[2]), int(p[3]))
            else:
                out[("join", int(p[1]))] = dict(zip(JOIN_FIELDS, (int(x) for x in p[2:])))
    return out
