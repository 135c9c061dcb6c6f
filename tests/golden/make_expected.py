"""Write the oracle's results for every request of the full-size batched
workload (16 tables, 448 selectivity + 64 join-frequency requests) and of the
served workload's 2,048-request pool.

Only `oracle/` and the `datagen/` recipes are used: each request's kept
blocks come from the oracle's sampler, their rows are regenerated on the host
by the counter-based generator, and the oracle counts on them (the definition
of the sampled predicate count, Sec. III-B and Eq. 2; the join-key
frequencies, NDV (Eq. 1) and sum f_R f_S (Eq. 3) from a sort of the sampled
keys).  The device path is never involved.

Output (text, one request per line, in the workload's own request order):
    sel  <i> <sampled_rows> <kept_blocks> <count_0> ... <count_{m-1}>
    join <j> <join_card> <ndv_R> <ndv_S> <n_R> <n_S> <f1_R> <f1_S> <f2_R> <f2_S>
preceded by a `fingerprint <sha256>` line naming the workload definition
(table sizes and ids, column laws, predicates, sampling specs), so a reader
can tell when the recipes have changed under a stored file.

Usage:  python tests/golden/make_expected.py [c4|c5] [--threads N]
The served pool shares its 64 join pairs with the batched workload, so the
c5 file reuses the c4 file's join lines (c4 must exist first).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import datagen  # noqa: E402
import oracle   # noqa: E402
from expected_io import FILES, JOIN_FIELDS, _table, fingerprint, load  # noqa: E402,F401


def workload(name: str):
    return datagen.config4() if name == "c4" else datagen.config5()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c4", "c5"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 8)
    a = ap.parse_args()
    w = workload(a.which)
    joins = {}
    if a.which == "c5":
        w4 = workload("c4")
        assert [_table(j.r) for j in w4.joins] == [_table(j.r) for j in w.joins]
        joins = {k[1]: v for k, v in load("c4", w4).items() if k[0] == "join"}
    lines = []
    t0 = time.time()
    for n, (kind, i) in enumerate(w.order):
        if kind == "sel":
            counts, sampled, kept = oracle.sel_request(w, i, nthreads=a.threads)
            lines.append("sel %d %d %d %s" % (i, sampled, kept, " ".join(str(int(c)) for c in counts)))
        else:
            r = joins.get(i) or oracle.join_request(w, i, nthreads=a.threads)
            joins[i] = r
            lines.append("join %d %s" % (i, " ".join(str(r[k]) for k in JOIN_FIELDS)))
        if n % 32 == 31:
            print("%s: %d / %d requests, %.0f s" % (a.which, n + 1, len(w.order), time.time() - t0), flush=True)
    tmp = FILES[a.which] + ".tmp"
    with open(tmp, "w") as f:
        f.write("fingerprint %s\n" % fingerprint(w))
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, FILES[a.which])
    print("wrote", FILES[a.which], "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
