"""The full-size served workload: 144 tables (170 GB) and 64 join pairs
resident, every one of the 2,048 pool requests submitted to a server at
once, each served result equal to the oracle's stored result
(tests/golden/c5_pool_expected.txt, written by make_expected.py from the
oracle alone)."""
import os
import sys

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import expected_io  # noqa: E402


def test_full_pool_served_equals_oracle():
    import torch

    import paper_2512_19750_amd as g
    torch.cuda.set_device(0)
    torch.cuda.empty_cache()            # the server allocates its workspace outside torch's cache
    dev = torch.device("cuda:0")
    w = datagen.config5()
    want = expected_io.load("c5", w)    # refuses a changed workload definition
    tabs, keys = datagen.materialise(w, dev)
    torch.cuda.synchronize()
    print("config 5 resident:", sum(c.numel() * c.element_size() for t in tabs for c in t) / 1e9, "GB", flush=True)
    reqs = []
    for kind, i in w.order:
        if kind == "sel":
            r = w.sel[i]
            t = w.tables[r.table]
            reqs.append(g.SelRequest(g.Table(tabs[r.table], t.table_id), r.preds, r.spec.seed, r.spec.rate,
                                     r.spec.block_rows))
        else:
            j = w.joins[i]
            kr, ks = keys[i]
            reqs.append(g.JoinRequest(g.Keys(kr, j.r.table_id, j.spec_r.seed, j.spec_r.rate, j.spec_r.block_rows),
                                      g.Keys(ks, j.s.table_id, j.spec_s.seed, j.spec_s.rate, j.spec_s.block_rows)))
    free_b, _ = torch.cuda.mem_get_info()
    srv = g.gace_server_create(0, max_inflight=3, max_batch=64, queue_capacity=4096,
                               workspace_bytes=int(min(48 << 30, free_b * 0.7)))
    try:
        tickets = [g.gace_server_submit(srv, q) for q in reqs]
        status = [g.gace_server_wait(srv, t, 300_000_000_000) for t in tickets]
        stats = g.gace_server_stats_get(srv)
    finally:
        g.gace_server_destroy(srv)
    assert status == [0] * len(reqs)
    assert stats["completed"] == len(reqs) and stats["batches"] > 1
    bad = []
    for (kind, i), q in zip(w.order, reqs):
        if kind == "join":
            got = q.result()
        else:
            c, n, b = q.result()
            got = (c.tolist(), n, b)
        if got != want[(kind, i)]:
            bad.append((kind, i))
    assert not bad, bad[:10]
    del tabs, keys
    torch.cuda.empty_cache()
