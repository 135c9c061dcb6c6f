"""Serving path on the GPU: requests submitted from several threads while other
batches run are admitted, batched and completed; every result equals the
request's plain-path result and the oracle's (alone == in the mix)."""
import threading

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2512_19750_amd as g
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = datagen.config4(scale=0.003, n_sel=80, n_join=10, seed_offset=11)
    tabs, keys = datagen.materialise(w, dev)
    return g, w, tabs, keys


def _req(g, w, tabs, keys, kind, i):
    if kind == "sel":
        r = w.sel[i]
        t = w.tables[r.table]
        return g.SelRequest(g.Table(tabs[r.table], t.table_id), r.preds, r.spec.seed, r.spec.rate, r.spec.block_rows)
    j = w.joins[i]
    kr, ks = keys[i]
    return g.JoinRequest(g.Keys(kr, j.r.table_id, j.spec_r.seed, j.spec_r.rate, j.spec_r.block_rows),
                         g.Keys(ks, j.s.table_id, j.spec_s.seed, j.spec_s.rate, j.spec_s.block_rows))


def _res(g, q):
    if isinstance(q, g.JoinRequest):
        return q.result()
    c, n, b = q.result()
    return (c.tolist(), n, b)


def test_served_results_equal_alone_and_oracle(env):
    g, w, tabs, keys = env
    order = list(w.order)
    # results alone (plain path)
    ctx = g.gace_create(0, 2 << 30)
    alone = {}
    try:
        for kind, i in order:
            q = _req(g, w, tabs, keys, kind, i)
            if kind == "sel":
                c, n, b = g.gace_probe_selectivity(ctx, q.table, q.preds, q.seed, q.rate, q.block_rows)
                alone[(kind, i)] = (c.tolist(), n, b)
            else:
                alone[(kind, i)] = g.gace_join_freq(ctx, q.R, q.S)
    finally:
        g.gace_destroy(ctx)
    # served: 4 submitting threads, small batches so several batches overlap
    srv = g.gace_server_create(0, max_inflight=3, max_batch=16, queue_capacity=1024, workspace_bytes=6 << 30)
    served = {}
    errors = []
    try:
        def worker(part):
            try:
                mine = []
                for kind, i in part:
                    q = _req(g, w, tabs, keys, kind, i)
                    mine.append(((kind, i), q, g.gace_server_submit(srv, q)))
                for key, q, t in mine:
                    st = g.gace_server_wait(srv, t, 60_000_000_000)
                    served[key] = (st, _res(g, q))
            except Exception as e:  # surfaced below
                errors.append(e)
        threads = [threading.Thread(target=worker, args=(order[k::4],)) for k in range(4)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        stats = g.gace_server_stats_get(srv)
    finally:
        g.gace_server_destroy(srv)
    assert not errors, errors
    assert stats["completed"] == len(order) and stats["batches"] >= 2
    # requests finish as their own scan or join does
    assert stats["completed_early"] > 0, stats
    for key in alone:
        st, res = served[key]
        assert st == 0, key
        assert res == alone[key], key
    # and every request against the oracle
    for kind, i in order:
        if kind == "sel":
            c, n, b = oracle.sel_request(w, i)
            assert alone[(kind, i)] == (c.tolist(), n, b), (kind, i)
        else:
            assert alone[(kind, i)] == oracle.join_request(w, i), (kind, i)


def test_probe_finishes_before_the_join_in_its_batch(env):
    """A small probe batched with a large join is done (results written, waiter
    woken) before the join: completion is per request, not per batch."""
    import torch
    g, w, tabs, keys = env
    dev = torch.device("cuda:0")
    r, s = datagen.join_pair(40_000_000, 10_000_000, 2_000_000, 77, 41, 42)
    kr = datagen.device_column(r.cols[0], r.n_rows, dev)
    ks = datagen.device_column(s.cols[0], s.n_rows, dev)
    big = [g.JoinRequest(g.Keys(kr, r.table_id, 5 + k, 1.0, 4096), g.Keys(ks, s.table_id, 6 + k, 1.0, 4096))
           for k in range(2)]
    kind, i = next(o for o in w.order if o[0] == "sel")
    small = _req(g, w, tabs, keys, kind, i)
    srv = g.gace_server_create(0, max_inflight=1, max_batch=64, queue_capacity=64, workspace_bytes=8 << 30)
    try:
        t_block = g.gace_server_submit(srv, big[0])        # occupies the only slot
        import time
        t_end = time.monotonic() + 30
        while g.gace_server_stats_get(srv)["batches"] < 1 and time.monotonic() < t_end:
            time.sleep(1e-4)
        t_join = g.gace_server_submit(srv, big[1])         # these two queue behind it
        t_small = g.gace_server_submit(srv, small)         # and form the next batch
        st_s, _, done_s = g.gace_server_wait_times(srv, t_small, 60_000_000_000)
        st_j, _, done_j = g.gace_server_wait_times(srv, t_join, 60_000_000_000)
        st_b, _, _ = g.gace_server_wait_times(srv, t_block, 60_000_000_000)
        stats = g.gace_server_stats_get(srv)
    finally:
        g.gace_server_destroy(srv)
    assert (st_s, st_j, st_b) == (0, 0, 0)
    assert stats["batches"] == 2, stats
    assert done_s < done_j, (done_s, done_j)
    c, n, b = oracle.sel_request(w, i)
    assert _res(g, small) == (c.tolist(), n, b)
    want = oracle.join_freq(kr.cpu().numpy(), r.table_id, 6, 1.0, 4096, ks.cpu().numpy(), s.table_id, 7, 1.0, 4096)
    assert big[1].result() == want


def test_server_rejects_invalid_and_oversized(env):
    g, w, tabs, keys = env
    srv = g.gace_server_create(0, max_inflight=1, max_batch=8, queue_capacity=8, workspace_bytes=512 << 20)
    try:
        import torch
        bad = g.SelRequest(g.Table(tabs[0], 100), [[(7, g.EQ, (1,))]])
        with pytest.raises(g.GaceError) as e:
            g.gace_server_submit(srv, bad)
        assert e.value.status == g.GACE_EINVAL
        big = torch.zeros(200_000_000, dtype=torch.int64, device="cuda")
        huge = g.JoinRequest(g.Keys(big, 1), g.Keys(big, 2))
        with pytest.raises(g.GaceError) as e:
            g.gace_server_submit(srv, huge)
        assert e.value.status == g.GACE_ENOMEM
        ok = _req(g, w, tabs, keys, "sel", 0)
        t = g.gace_server_submit(srv, ok)
        st, t_sub, t_done = g.gace_server_wait_times(srv, t, 60_000_000_000)
        assert st == 0 and 0 < t_sub <= t_done
        st = g.gace_server_stats_get(srv)
        assert st["rejected"] == 2 and st["completed"] == 1
        del big
    finally:
        g.gace_server_destroy(srv)


def test_tracing_records_every_item(env):
    g, w, tabs, keys = env
    ctx = g.gace_create(0, 2 << 30)
    try:
        reqs = [_req(g, w, tabs, keys, k, i) for k, i in w.order[:40]]
        g.gace_set_trace(ctx, True)
        g.gace_batch_run(ctx, reqs)
        tr, tpu = g.gace_get_trace(ctx)
        assert len(tr) > 0 and tpu > 0
        assert np.all(tr["t_end"] >= tr["t_ready"]) and np.all(tr["t_ready"] >= tr["t_begin"])
        assert set(np.unique(tr["kind"]).tolist()) <= {1, 2, 3, 4, 5, 6, 7, 8}
        assert np.all(tr["xcc"] < 16)
    finally:
        g.gace_destroy(ctx)


def test_open_loop_stream_equals_plain(env):
    """The benchmark's open-loop Poisson driver: every served result equals the
    request's plain-path result, and latencies are measured for the counted
    arrivals."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    g, w, tabs, keys = env
    reqs = [_req(g, w, tabs, keys, k, i) for k, i in w.order]
    kinds = [k for k, _ in w.order]
    ctx = g.gace_create(0, 2 << 30)
    expect = []
    try:
        for q in reqs:
            if isinstance(q, g.JoinRequest):
                r = g.gace_join_freq(ctx, q.R, q.S)
                expect.append(tuple(r[f] for f in bench.JOIN_FIELDS))
            else:
                c, n, b = g.gace_probe_selectivity(ctx, q.table, q.preds, q.seed, q.rate, q.block_rows)
                expect.append((tuple(int(x) for x in c), n, b))
    finally:
        g.gace_destroy(ctx)
    arr, keep = g.make_requests(reqs)
    r = bench.serve_point(g, arr, expect, kinds, 400.0,
                          dict(max_inflight=2, max_batch=16, queue_capacity=512, workspace_bytes=3 << 30),
                          seed=5, duration_s=2.0, warm_s=0.2, ring=1024)
    assert r["mismatches"] == 0 and r["rejected_busy"] == 0
    assert r["counted"] > 0 and r["p99_ms"] >= r["p50_ms"] > 0


def test_two_waiters_on_one_ticket(env):
    """Two threads wait for the same ticket: one collects it, the other gets
    GACE_EINVAL instead of blocking on a re-created entry."""
    g, w, tabs, keys = env
    kind, i = next(o for o in w.order if o[0] == "sel")
    q = _req(g, w, tabs, keys, kind, i)
    srv = g.gace_server_create(0, max_inflight=1, max_batch=4, queue_capacity=16, workspace_bytes=1 << 30)
    out = []
    try:
        t = g.gace_server_submit(srv, q)

        def waiter():
            try:
                out.append(("ok", g.gace_server_wait(srv, t, 30_000_000_000)))
            except g.GaceError as e:
                out.append(("err", e.status))
        ths = [threading.Thread(target=waiter) for _ in range(2)]
        for th in ths:
            th.start()
        for th in ths:
            th.join(60)
        assert not any(th.is_alive() for th in ths)
    finally:
        g.gace_server_destroy(srv)
    assert sorted(out) == [("err", g.GACE_EINVAL), ("ok", 0)], out
