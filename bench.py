#!/usr/bin/env python3
"""Benchmark: the batched uneven probe workload on one MI355X.

A step is one gace_batch_run of the whole request list: 448 selectivity
requests (1-32 conjunctive predicates each, sampling rate log-uniform in
[0.1 %, 100 %]) over 16 resident tables (log-uniform 10^6..5x10^8 rows x 4
int32 columns) and 64 join-key frequency probes (Zipf R / uniform S, scaled
0.01..1 of 200M + 50M keys, rate 1 or 0.05), in one persistent, graph-
replayed launch.  Inputs are generated in device memory before timing.

Prints one JSON line: rows*predicates/s of the batch, HBM roofline of the
persistent kernel, the plain one-launch-per-request path on the same
requests, per-request latency of that path, and the CPU oracle on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
CSRC = os.path.join(ROOT, "paper_2512_19750_amd", "csrc")
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("kernels.hip", "plan.h", "compile.cpp")]


def kernel_hash() -> str:
    """Hash of the sources that decide what the kernels read and write."""
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counters_path(kernel: str) -> str:
    return os.path.join(ROOT, "profiles", "%s_c4_counters.md" % kernel)


def stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None)."""
    path = counters_path(kernel)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = None
    t = None
    for line in txt.splitlines():
        if line.startswith("kernel_source_sha256_16:"):
            h = line.split(":", 1)[1].strip()
        if line.startswith("hbm_bytes_per_launch:"):
            t = float(line.split(":", 1)[1].strip())
    if h != kernel_hash() or t is None:
        return None
    return t


def build_requests(g, w, tabs, keys):
    out = []
    for kind, i in w.order:
        if kind == "sel":
            r = w.sel[i]
            t = w.tables[r.table]
            out.append(g.SelRequest(g.Table(tabs[r.table], t.table_id), r.preds, r.spec.seed, r.spec.rate,
                                    r.spec.block_rows))
        else:
            j = w.joins[i]
            kr, ks = keys[i]
            out.append(g.JoinRequest(g.Keys(kr, j.r.table_id, j.spec_r.seed, j.spec_r.rate, j.spec_r.block_rows),
                                     g.Keys(ks, j.s.table_id, j.spec_s.seed, j.spec_s.rate, j.spec_s.block_rows)))
    return out


def cpu_baseline(w, budget_rows_preds: float, nthreads: int):
    """Oracle rows*predicates/s on a bounded sample: selectivity requests taken
    in batch order until the sample holds ~budget rows*predicates."""
    import numpy as np

    import datagen
    import oracle
    picked, total = [], 0
    for kind, i in w.order:
        if kind != "sel":
            continue
        r = w.sel[i]
        t = w.tables[r.table]
        kb = oracle.kept_blocks(t.n_rows, r.spec.seed, t.table_id, r.spec.rate, r.spec.block_rows)
        rows = sum(min(t.n_rows, (int(b) + 1) * r.spec.block_rows) - int(b) * r.spec.block_rows for b in kb)
        rp = rows * len(r.preds)
        if rp == 0 or total + rp > budget_rows_preds:
            continue
        picked.append((i, kb))
        total += rp
        if total > 0.9 * budget_rows_preds:
            break
    secs, rp_done, rows_done = 0.0, 0, 0
    for i, kb in picked:
        r = w.sel[i]
        t = w.tables[r.table]
        spans = oracle.merge_spans([(int(b) * r.spec.block_rows, min(t.n_rows, (int(b) + 1) * r.spec.block_rows))
                                    for b in kb])
        cols = [np.concatenate([datagen.host_column(c, e - b, row0=b, nthreads=nthreads) for b, e in spans])
                for c in t.cols]
        t0 = time.perf_counter()
        counts, sampled, _ = oracle.probe_selectivity(cols, [c.dtype for c in t.cols], t.table_id, r.preds,
                                                      0, 1.0, 1 << 20, nthreads)
        secs += time.perf_counter() - t0
        rp_done += sampled * len(r.preds)
        rows_done += sampled
        del cols
    return dict(value=rp_done / secs if secs > 0 else None, unit="rows*predicates/s", cores=nthreads,
                kind="oracle", seconds=round(secs, 3),
                sample="%d of %d selectivity requests in batch order (%d sampled rows, %.3g rows*predicates); "
                       "kept-block rows regenerated on the host, counting timed"
                       % (len(picked), len(w.sel), rows_done, rp_done))


# ---------------------------------------------------------------- serving
def gate_measurement(g, ctx, sel_reqs, sel_obs):
    """The decision layer on the measured plain-path probes: the cost model
    fitted to their latencies (how well it predicts them), the cost of a gate
    evaluation, and the latency of a probe answered from the result cache
    against the probe itself."""
    m = g.gace_cost_create(0.85, 4096)
    try:
        feats = []
        for q, (nrow, ms) in zip(sel_reqs, sel_obs):
            _, row_bytes, terms = g.gace_cost_features_of(q)
            feats.append((nrow, row_bytes, terms, ms))
            g.gace_cost_observe(m, nrow, row_bytes, terms, ms)
        coef, n_obs = g.gace_cost_coef(m)
        rel = sorted(abs(g.gace_cost_predict(m, n, b, t) - ms) / ms for n, b, t, ms in feats)
    finally:
        g.gace_cost_destroy(m)
    t0 = time.perf_counter()
    k = 20000
    for i in range(k):
        g.gace_gate_evaluate(ndv=(1000.0, 700.0 + i % 600), sel=(0.1, i % 300, 1000), pcs=(i % 50, 50, 60, 1000))
    eval_us = (time.perf_counter() - t0) / k * 1e6
    c = g.gace_cache_create(1 << 20)
    cold, warm = [], []
    try:
        for q in sel_reqs[:64]:
            for lst in (cold, warm):
                s = time.perf_counter()
                g.gace_probe_selectivity_cached(ctx, c, q.table, q.preds, q.seed, q.rate, q.block_rows)
                lst.append((time.perf_counter() - s) * 1e3)
        st = g.gace_cache_stats_get(c)
    finally:
        g.gace_cache_destroy(c)
    return {"cost_model": {"coef_ms": [coef[0], coef[1], coef[2]],
                           "terms": ["fixed", "per byte read", "per row-term"], "observations": n_obs,
                           "rel_error_p50": round(rel[len(rel) // 2], 4),
                           "rel_error_p90": round(rel[int(0.9 * (len(rel) - 1))], 4)},
            "gate_eval_us": round(eval_us, 3),
            "cache": {"probe_ms_p50": round(_pct(cold, 0.5), 4), "hit_ms_p50": round(_pct(warm, 0.5), 4),
                      "hits": st["hits"], "misses": st["misses"]}}


def _pct(xs, q):
    if not xs:
        return None
    xs = sorted(xs)
    return xs[min(len(xs) - 1, max(0, int(math.ceil(q * len(xs))) - 1))]


def serve_point(g, pool_arr, expect, kinds, qps, cfg, seed, duration_s=10.0, max_req=20000, warm_s=1.0,
                ring=8192):
    """Open-loop Poisson arrivals at `qps` for duration_s (or max_req
    requests), each request drawn uniformly from the pool.  Latency = the
    server's completion time - the scheduled arrival time; arrivals in the
    first warm_s seconds are not counted.  Every served result is compared
    with the pool entry's plain-path result."""
    import ctypes
    import queue as _q
    import threading

    import numpy as np
    rng = np.random.default_rng(seed)
    n = int(min(max_req, qps * duration_s))
    arrivals = np.cumsum(rng.exponential(1.0 / qps, n))
    picks = rng.integers(0, len(kinds), n)
    ring_arr = (g.gace_request * ring)()
    counts = np.zeros((ring, 32), dtype=np.uint64)
    infos = (g.gace_probe_info * ring)()
    jres = (g.gace_join_result * ring)()
    cptr = [counts[i].ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) for i in range(ring)]
    iptr = [ctypes.pointer(infos[i]) for i in range(ring)]
    jptr = [ctypes.pointer(jres[i]) for i in range(ring)]
    srv = g.gace_server_create(0, **cfg)
    work = _q.Queue()
    lat, bad, done_t, seen = [], [0], [], [0]

    def waiter():
        while True:
            item = work.get()
            if item is None:
                return
            i, slot, t, sched = item
            if t is None:          # rejected with EBUSY: nothing to read
                seen[0] = i + 1
                continue
            st, _, t_done = g.gace_server_wait_times(srv, t, -1)
            p = int(picks[i])
            if kinds[p] == "join":
                o = jres[slot]
                got = (int(o.join_card), int(o.ndv_R), int(o.ndv_S), int(o.n_R), int(o.n_S))
            else:
                k = len(expect[p][0])
                got = (tuple(int(x) for x in counts[slot][:k]), int(infos[slot].sampled_rows),
                       int(infos[slot].kept_blocks))
            if st != 0 or got != expect[p]:
                bad[0] += 1
            if arrivals[i] >= warm_s:
                lat.append((t_done - sched) / 1e6)
                done_t.append(t_done)
            seen[0] = i + 1

    th = threading.Thread(target=waiter)
    th.start()
    busy = 0
    t0 = time.monotonic_ns() + 20_000_000
    try:
        for i in range(n):
            sched = t0 + int(arrivals[i] * 1e9)
            while True:
                now = time.monotonic_ns()
                if now >= sched:
                    break
                if sched - now > 300_000:
                    time.sleep((sched - now - 200_000) / 1e9)
            slot = i % ring
            while seen[0] + ring <= i and th.is_alive():   # slot's previous result not read yet
                time.sleep(1e-4)
            p = int(picks[i])
            r = ring_arr[slot]
            ctypes.memmove(ctypes.byref(r), ctypes.byref(pool_arr[p]), ctypes.sizeof(g.gace_request))
            if kinds[p] == "join":
                r.join = jptr[slot]
            else:
                r.counts = cptr[slot]
                r.info = iptr[slot]
            try:
                t = g.gace_server_submit_raw(srv, ctypes.byref(r))
            except g.GaceError as e:
                if e.status != g.GACE_EBUSY:
                    raise
                busy += 1
                t = None
            work.put((i, slot, t, sched))
    finally:
        work.put(None)
        th.join()
        stats = g.gace_server_stats_get(srv)
        g.gace_server_destroy(srv)
    t_first = t0 + int(warm_s * 1e9)
    span = (max(done_t) - t_first) / 1e9 if done_t else 0.0
    return dict(qps=qps, offered=n, counted=len(lat), rejected_busy=busy, mismatches=bad[0],
                p50_ms=round(_pct(lat, 0.50), 3) if lat else None, p99_ms=round(_pct(lat, 0.99), 3) if lat else None,
                throughput_rps=round(len(lat) / span, 1) if span > 0 else None, batches=stats["batches"],
                workspace_peak=stats["workspace_peak"])


def serve_main(args):
    import torch

    import datagen
    import paper_2512_19750_amd as g
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_setup = time.time()
    w = datagen.config5(scale=args.scale)
    tabs, keys = datagen.materialise(w, dev)
    torch.cuda.synchronize()
    resident = sum(c.numel() * c.element_size() for t in tabs for c in t) + \
        sum(k.numel() * 8 for pair in keys for k in pair)
    print("[serve] %d tables + %d join pairs, %.1f GB resident, %.1fs" % (len(tabs), len(keys), resident / 1e9,
                                                                       time.time() - t_setup),
          file=sys.stderr, flush=True)
    pool = build_requests(g, w, tabs, keys)
    kinds = [k for k, _ in w.order]
    pool_arr, keep = g.make_requests(pool)
    # plain-path results of every pool entry (each served result must equal them)
    free_b, _ = torch.cuda.mem_get_info()
    ctx = g.gace_create(0, int(min(24 << 30, free_b * 0.8)))
    t0 = time.time()
    expect, plain_lat = [], []
    for q in pool:
        s0 = time.perf_counter()
        if isinstance(q, g.JoinRequest):
            r = g.gace_join_freq(ctx, q.R, q.S)
            expect.append((r["join_card"], r["ndv_R"], r["ndv_S"], r["n_R"], r["n_S"]))
        else:
            c, nrow, nblk = g.gace_probe_selectivity(ctx, q.table, q.preds, q.seed, q.rate, q.block_rows)
            expect.append((tuple(int(x) for x in c), nrow, nblk))
        plain_lat.append((time.perf_counter() - s0) * 1e3)
    g.gace_destroy(ctx)
    plain_s = time.time() - t0
    print("[serve] plain path over the pool: %.1fs (%.1f req/s)" % (plain_s, len(pool) / plain_s), file=sys.stderr,
          flush=True)
    free_b, _ = torch.cuda.mem_get_info()
    ws = int(min(args.serve_workspace_gb * (1 << 30), free_b * 0.8))
    modes = {
        "batched": dict(max_inflight=3, max_batch=64, queue_capacity=4096, workspace_bytes=ws),
        "fifo_one_launch_per_request": dict(max_inflight=1, max_batch=1, queue_capacity=4096,
                                            workspace_bytes=ws // 3),
    }
    points = []
    for qps in [int(x) for x in args.serve_qps.split(",")]:
        for name, cfg in modes.items():
            r = serve_point(g, pool_arr, expect, kinds, qps, cfg, seed=S_SERVE + qps,
                            duration_s=args.serve_seconds)
            r["mode"] = name
            points.append(r)
            print("[serve] %s" % json.dumps(r), file=sys.stderr, flush=True)
    out = {
        "metric": "served probe latency (completion - scheduled Poisson arrival) and throughput",
        "unit": "ms",
        "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic (seeded counter-based generator, generated in HBM)",
        "config": {"workload": "C5 served probe stream: %d tables of config 4's size law + 64 join pairs, "
                               "%.1f GB resident, pool of %d requests from config 4's mix (%d joins)%s"
                               % (len(tabs), resident / 1e9, len(pool), kinds.count("join"),
                                  "" if args.scale == 1.0 else " (scale %g)" % args.scale),
                   "arrivals": "open-loop Poisson, %gs or 20000 requests per point, first 1s not counted"
                               % args.serve_seconds},
        "plain_path_pool": {"seconds": round(plain_s, 3),
                            "latency_ms_p50": round(_pct(plain_lat, 0.5), 4),
                            "latency_ms_p99": round(_pct(plain_lat, 0.99), 4)},
        "points": points,
    }
    print(json.dumps(out))


S_SERVE = 0x2512197500 + 40
S_H2D = 0x2512197500 + 50


def h2d_main(args):
    """Exp. A on MI355X: a selectivity probe of a host-resident table, split
    into sampler, gather, host-to-device copy, kernel, download and reduction,
    for sample sizes N from 1e4 to the whole table, moving only the referenced
    columns (key-only) or every column (full row); the same probe of the table
    resident in HBM is timed beside it."""
    import torch

    import datagen
    import paper_2512_19750_amd as g
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n_rows = int(args.h2d_rows)
    t = datagen.uniform_i32_table(n_rows, 4, S_H2D, table_id=1)
    t0 = time.time()
    host = datagen.host_table(t, nthreads=16)
    resident = [torch.from_numpy(c).to(dev) for c in host]
    torch.cuda.synchronize()
    print("[h2d] table %d rows x 4 int32 (%.2f GB) in host memory, %.1fs" % (n_rows, 16 * n_rows / 1e9,
                                                                         time.time() - t0), file=sys.stderr,
          flush=True)
    pred = [[(0, g.RANGE, (100, 300)), (1, g.RANGE, (0, 500))]]     # key-only: 2 of 4 columns
    ctx = g.gace_create(0, 8 << 30)
    points = []
    try:
        for n_target in [float(x) for x in args.h2d_n.split(",")]:
            rate = min(1.0, n_target / n_rows)
            row = {"n_target": n_target, "rate": rate}
            for mode in ("key_only", "full_row"):
                runs = []
                for rep in range(1 + args.h2d_reps):
                    c, n, k, st = g.gace_probe_selectivity_host(ctx, host, 1, pred, S_H2D, rate, 4096,
                                                                key_only=(mode == "key_only"))
                    if rep:
                        runs.append(st)
                med = {key: sorted(r[key] for r in runs)[len(runs) // 2]
                       for key in ("total_ms", "sample_ms", "gather_ms", "h2d_ms", "kernel_ms", "d2h_ms",
                                   "reduce_ms")}
                med = {key: round(v, 4) for key, v in med.items()}
                med["h2d_bytes"] = runs[0]["h2d_bytes"]
                med["h2d_gbps"] = round(med["h2d_bytes"] / (med["h2d_ms"] * 1e6), 2) if med["h2d_ms"] else None
                med["chunks"] = runs[0]["chunks"]
                row[mode] = med
                row["sampled_rows"], row["count"] = n, int(c[0])
            lat = []
            for rep in range(1 + args.h2d_reps):
                s0 = time.perf_counter()
                c2, n2, _ = g.gace_probe_selectivity(ctx, g.Table(resident, 1), pred, S_H2D, rate, 4096)
                if rep:
                    lat.append((time.perf_counter() - s0) * 1e3)
            assert int(c2[0]) == row["count"] and n2 == row["sampled_rows"]
            row["resident_ms"] = round(sorted(lat)[len(lat) // 2], 4)
            points.append(row)
            print("[h2d] %s" % json.dumps(row), file=sys.stderr, flush=True)
    finally:
        g.gace_destroy(ctx)
    print(json.dumps({"metric": "host-resident probe time decomposition (Exp. A), key-only vs full row",
                      "unit": "ms", "n_gpus": 1, "table_rows": n_rows, "columns": "4 x int32, predicate on 2",
                      "data": "synthetic (seeded counter-based generator)", "points": points}))


S_EST = 0x2512197500 + 60
S_ZONE = 0x2512197500 + 70


def zone_main(args):
    """Zone maps on MI355X: build time of the per-zone min / max of a table,
    and selectivity probes with and without zone pruning on the table as
    generated and clustered by the filtered column."""
    import torch

    import datagen
    import paper_2512_19750_amd as g
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n_rows = int(args.zone_rows)
    t = datagen.uniform_i32_table(n_rows, 4, S_ZONE, table_id=7, lo=0, hi=1_000_000)
    cols = datagen.device_table(t, dev)
    order = torch.argsort(cols[0], stable=True)
    layouts = {"random": cols, "clustered": [c[order].contiguous() for c in cols]}
    del order
    torch.cuda.synchronize()
    preds = {"1% range on c0": [[(0, g.RANGE, (500_000, 510_000))]],
             "1% range on c0 and c1 < 50%": [[(0, g.RANGE, (500_000, 510_000)), (1, g.RANGE, (0, 500_000))]],
             "16 point lookups on c0": [[(0, g.EQ, (v,))] for v in range(1000, 1_000_000, 62_437)]}
    ctx = g.gace_create(0, 8 << 30)
    out = {"metric": "zone-map build and pruned probe time", "n_gpus": 1, "table_rows": n_rows,
           "columns": "4 x int32 U[0, 1e6)", "build": {}, "points": []}

    def timed(f, reps=5):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            s0 = time.perf_counter()
            r = f()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - s0) * 1e3)
        return sorted(ts)[len(ts) // 2], r

    try:
        for layout, tcols in layouts.items():
            tab = g.Table(tcols, 7)
            ms, zm = timed(lambda: g.gace_zonemap_build(ctx, tab), reps=1)
            g.gace_zonemap_destroy(zm)
            ms, zm = timed(lambda: g.gace_zonemap_build(ctx, tab), reps=1)
            out["build"][layout] = {"ms": round(ms, 4), "gbps": round(16 * n_rows / (ms * 1e6), 1)}
            try:
                for name, ps in preds.items():
                    for rate in (1.0, 0.01):
                        m0, r0 = timed(lambda: g.gace_probe_selectivity(ctx, tab, ps, S_ZONE, rate, 4096))
                        m1, r1 = timed(lambda: g.gace_probe_selectivity_zm(ctx, tab, zm, ps, S_ZONE, rate, 4096))
                        assert r0[0].tolist() == r1[0].tolist() and r0[1:] == r1[1:3]
                        row = {"layout": layout, "predicates": name, "rate": rate, "plain_ms": round(m0, 4),
                               "zone_ms": round(m1, 4), "zones_skipped": r1[3],
                               "zones": g.gace_zonemap_info(zm), "speedup": round(m0 / m1, 2)}
                        out["points"].append(row)
                        print("[zone] %s" % json.dumps(row), file=sys.stderr, flush=True)
            finally:
                g.gace_zonemap_destroy(zm)
    finally:
        g.gace_destroy(ctx)
    print(json.dumps(out))




def est_main(args):
    """Exp. B on MI355X: spread of the sampled estimates of sel(A AND B) and of
    PCS across sampling seeds (Est.CV) against the probing budget, for block
    sampling (4096-row blocks) and row sampling, on the table as generated
    and on the same table clustered by A's column.  Each (layout, block size,
    budget) point is one batched launch of `seeds` probes."""
    import torch

    import datagen
    import paper_2512_19750_amd as g
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n_rows = int(args.est_rows)
    t = datagen.config2_table(n_rows)
    c0 = datagen.device_column(t.cols[0], n_rows, dev)
    c1 = datagen.device_column(t.cols[1], n_rows, dev)       # c0 + U{-50..50}: correlated with c0
    order = torch.argsort(c0, stable=True)
    layouts = {"random": [c0, c1], "clustered": [c0[order].contiguous(), c1[order].contiguous()]}
    del order
    torch.cuda.synchronize()
    A = [(0, g.RANGE, (1000, 1100))]
    B = [(1, g.RANGE, (1000, 1100))]
    preds = [A, B, A + B]
    ctx = g.gace_create(0, 8 << 30)
    g.gace_set_graph(ctx, True)
    points = []
    try:
        truth = g.gace_probe_selectivity(ctx, g.Table(layouts["random"], 2), preds, 0, 1.0, 4096)
        ca, cb, cab = (int(x) for x in truth[0])
        sel_true = cab / n_rows
        pcs_true = cab * n_rows / (ca * cb)
        print("[est] truth: c_a %d c_b %d c_ab %d of %d rows: sel %.3e PCS %.3f" % (ca, cb, cab, n_rows, sel_true,
                                                                                  pcs_true), file=sys.stderr,
              flush=True)
        for layout, cols in layouts.items():
            tab = g.Table(cols, 2)
            for brows in (4096, 1):
                for rate in [float(x) for x in args.est_rates.split(",")]:
                    reqs = [g.SelRequest(tab, preds, S_EST + k, rate, brows) for k in range(args.est_seeds)]
                    arr = g.make_requests(reqs)
                    g.gace_batch_run(ctx, reqs, prepared=arr)              # warm
                    t0 = time.perf_counter()
                    g.gace_batch_run(ctx, reqs, prepared=arr)
                    ms = (time.perf_counter() - t0) * 1e3
                    sel, pcs, rows = [], [], []
                    for q in reqs:
                        c, n, _ = q.result()
                        a_, b_, ab_ = (int(x) for x in c)
                        rows.append(n)
                        if n:
                            sel.append(ab_ / n)
                        if a_ and b_:
                            pcs.append(ab_ * n / (a_ * b_))
                    def cv(x):
                        m = float(np.mean(x)) if x else math.nan
                        return (float(np.std(x, ddof=1)) / m) if len(x) > 1 and m else math.nan, m
                    cv_sel, m_sel = cv(sel)
                    cv_pcs, m_pcs = cv(pcs)
                    row = {"layout": layout, "block_rows": brows, "rate": rate, "seeds": args.est_seeds,
                           "mean_sampled_rows": round(float(np.mean(rows)), 1),
                           "sel_cv": round(cv_sel, 4), "sel_bias": round(m_sel / sel_true - 1, 4),
                           "pcs_cv": round(cv_pcs, 4) if not math.isnan(cv_pcs) else None,
                           "pcs_bias": round(m_pcs / pcs_true - 1, 4) if pcs else None,
                           "pcs_defined": len(pcs), "batch_ms": round(ms, 3)}
                    points.append(row)
                    print("[est] %s" % json.dumps(row), file=sys.stderr, flush=True)
    finally:
        g.gace_destroy(ctx)
    print(json.dumps({"metric": "Est.CV of sel(A and B) and PCS across sampling seeds vs budget (Exp. B)",
                      "n_gpus": 1, "table_rows": n_rows, "data": "synthetic: c0 Zipf(1.1) over [0, 1e6), "
                      "c1 = c0 + U{-50..50}; A = c0 in [1000, 1100), B = c1 in [1000, 1100)",
                      "truth": {"sel": sel_true, "pcs": pcs_true}, "points": points}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink every size (tests only)")
    ap.add_argument("--plain", type=int, default=1, help="also time the one-launch-per-request path")
    ap.add_argument("--cpu-budget", type=float, default=1.2e10, help="rows*predicates of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2512_19750_amd", "tuned_schedules.jsonl"))
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="only copy this many bytes device-to-device 3 times (counter calibration) and exit")
    ap.add_argument("--serve", action="store_true",
                    help="run the served probe stream (config 5) instead of the batch benchmark")
    ap.add_argument("--serve-qps", default="100,200,500,1000,2000,5000")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-workspace-gb", type=float, default=60.0)
    ap.add_argument("--serve-point-qps", type=float, default=1000.0,
                    help="batch benchmark: also serve its requests at this Poisson rate (0: skip)")
    ap.add_argument("--serve-point-seconds", type=float, default=5.0)
    ap.add_argument("--h2d", action="store_true",
                    help="run the host-resident table decomposition (Exp. A) instead of the batch benchmark")
    ap.add_argument("--h2d-rows", type=float, default=1e8)
    ap.add_argument("--h2d-n", default="1e4,1e5,1e6,1e7,1e8")
    ap.add_argument("--h2d-reps", type=int, default=3)
    ap.add_argument("--est", action="store_true",
                    help="run the estimate-stability sweep (Exp. B) instead of the batch benchmark")
    ap.add_argument("--est-rows", type=float, default=1e8)
    ap.add_argument("--est-rates", default="0.0005,0.002,0.01,0.05")
    ap.add_argument("--est-seeds", type=int, default=64)
    ap.add_argument("--zone", action="store_true",
                    help="run the zone-map build and pruned-probe measurement instead of the batch benchmark")
    ap.add_argument("--zone-rows", type=float, default=4e8)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the probe on a single MI355X "
              "(multi-GPU sharding is a design note, not a code path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve_main(args)
        return
    if args.h2d:
        h2d_main(args)
        return
    if args.est:
        est_main(args)
        return
    if args.zone:
        zone_main(args)
        return

    import torch

    import datagen
    import paper_2512_19750_amd as g

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calib_copy:
        src = torch.ones(args.calib_copy // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": args.calib_copy}))
        return
    t_setup = time.time()
    w = datagen.config4(scale=args.scale)
    tabs, keys = datagen.materialise(w, dev)
    torch.cuda.synchronize()
    resident = sum(c.numel() * c.element_size() for t in tabs for c in t) + \
        sum(k.numel() * 8 for pair in keys for k in pair)
    print("[bench] generated %d tables + %d join pairs, %.1f GB resident, %.1fs"
          % (len(tabs), len(keys), resident / 1e9, time.time() - t_setup), file=sys.stderr, flush=True)

    free_b, _ = torch.cuda.mem_get_info()
    ws = int(min(free_b * 0.6, 48 << 30))
    ctx = g.gace_create(0, ws)
    reqs = build_requests(g, w, tabs, keys)
    prepared = g.make_requests(reqs)
    # the timed region launches directly (below), so the schedule is tuned
    # in that launch mode
    g.gace_set_graph(ctx, False)
    if args.autotune:
        t0 = time.time()
        g.gace_autotune(ctx, reqs, args.tune_cache)
        print("[bench] schedule %s (%.1fs)" % (g.gace_get_schedule(ctx), time.time() - t0), file=sys.stderr,
              flush=True)
    # timed region: direct launches, so that HIP events bracket each kernel on
    # its own stream (scan kernel on the call's stream, join kernel on the side
    # stream); results are identical to graph replay, which is timed after
    g.gace_set_graph(ctx, False)
    for _ in range(args.warmup):
        g.gace_batch_run(ctx, reqs, prepared=prepared)
    torch.cuda.synchronize()
    kms, sms, jms, cms = [], [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.gace_batch_run(ctx, reqs, prepared=prepared)
        kms.append(g.gace_last_batch_stats(ctx)["kernel_ms"])
        ks = g.gace_last_kernel_stats(ctx)
        sms.append(ks["scan_ms"])
        jms.append(ks["join_ms"])
        cms.append(ks["compile_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = g.gace_last_batch_stats(ctx)
    ms_step = wall / args.steps * 1e3
    rows_preds = st["rows_preds"]
    value = rows_preds / (wall / args.steps)
    kernel_ms = sum(kms) / len(kms)
    # the join stage is the partitioning kernel followed by the aggregation
    # kernel on one stream; its events bracket both
    per_kernel = {
        "gace_scan_kernel": dict(ms=sum(sms) / len(sms), alg_bytes=ks["scan_alg_bytes"]),
        "gace_join_stage": dict(ms=sum(jms) / len(jms), alg_bytes=ks["join_alg_bytes"],
                                kernels=["gace_join_kernel", "gace_agg_kernel"]),
    }
    for k in per_kernel.values():
        k["achieved_gbps"] = k["alg_bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0
    dominant = max(per_kernel, key=lambda k: per_kernel[k]["ms"])
    dk = per_kernel[dominant]
    achieved = dk["achieved_gbps"]
    traffic = stored_traffic(dominant)
    # graph replay of the same batch (the batched path's default)
    g.gace_set_graph(ctx, True)
    g.gace_batch_run(ctx, reqs, prepared=prepared)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.gace_batch_run(ctx, reqs, prepared=prepared)
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) / args.steps * 1e3
    sel_rows = 0
    join_keys = 0
    for q in reqs:
        if isinstance(q, g.JoinRequest):
            r = q.result()
            join_keys += r["n_R"] + r["n_S"]
        else:
            sel_rows += q.result()[1]
    compile_ms = sum(cms) / len(cms)
    print("[bench] batch %.2f ms/step (host compile %.2f ms, kernels %.2f ms: scan %.2f, join %.2f; graph replay "
          "%.2f ms/step), %.3g rows*preds/s" % (ms_step, compile_ms, kernel_ms, per_kernel["gace_scan_kernel"]["ms"],
                                               per_kernel["gace_join_stage"]["ms"], graph_ms, value),
          file=sys.stderr, flush=True)

    plain = None
    gate = None
    expect = []
    if args.plain:
        lat = []
        sel_obs = []                      # (sampled rows, row bytes, terms, ms) of each selectivity probe
        t0 = time.perf_counter()
        for q in reqs:
            s = time.perf_counter()
            if isinstance(q, g.JoinRequest):
                r = g.gace_join_freq(ctx, q.R, q.S)
                expect.append((r["join_card"], r["ndv_R"], r["ndv_S"], r["n_R"], r["n_S"]))
            else:
                c, nrow, nblk = g.gace_probe_selectivity(ctx, q.table, q.preds, q.seed, q.rate, q.block_rows)
                expect.append((tuple(int(x) for x in c), nrow, nblk))
            lat.append((time.perf_counter() - s) * 1e3)
            if not isinstance(q, g.JoinRequest):
                sel_obs.append((nrow, lat[-1]))
        plain_s = time.perf_counter() - t0
        lat.sort()
        plain = dict(ms_per_batch=round(plain_s * 1e3, 3), batched_speedup=round(plain_s * 1e3 / ms_step, 3),
                     latency_ms_p50=round(lat[len(lat) // 2], 4),
                     latency_ms_p99=round(lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)], 4))
        print("[bench] plain path %.1f ms (x%.2f)" % (plain_s * 1e3, plain["batched_speedup"]), file=sys.stderr,
              flush=True)
        gate = gate_measurement(g, ctx, [q for q in reqs if not isinstance(q, g.JoinRequest)], sel_obs)
        print("[bench] gate %s" % json.dumps(gate), file=sys.stderr, flush=True)
    sched = g.gace_get_schedule(ctx)
    g.gace_destroy(ctx)
    # served: the same requests arriving as an open-loop Poisson stream
    served = None
    if args.plain and args.serve_point_qps > 0:
        kinds = ["join" if isinstance(q, g.JoinRequest) else "sel" for q in reqs]
        served = serve_point(g, prepared[0], expect, kinds, args.serve_point_qps,
                             dict(max_inflight=3, max_batch=64, queue_capacity=4096, workspace_bytes=ws),
                             seed=S_SERVE, duration_s=args.serve_point_seconds)
        print("[bench] served %s" % json.dumps(served), file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        nthreads = min(os.cpu_count() or 1, 16)
        cpu = cpu_baseline(w, args.cpu_budget * args.scale, nthreads)
        print("[bench] oracle %.3g rows*preds/s on %d threads (%.1fs)" % (cpu["value"] or 0, nthreads,
                                                                         cpu["seconds"]), file=sys.stderr,
              flush=True)

    out = {
        "metric": "sampled rows*predicates/s (batched probe), with HBM GB/s, batched-vs-plain and p99 probe latency",
        "value": value,
        "unit": "rows*predicates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32,int64",
        "data": "synthetic (seeded counter-based generator, generated in HBM)",
        "config": {
            "workload": "C4 batched uneven probes: 448 selectivity requests (1-32 conjunctive predicates, "
                        "rate log-uniform 0.1-100%%, 4096-row blocks) over 16 tables of log-uniform 1e6-5e8 rows "
                        "x 4 int32 columns + 64 join-key frequency probes (Zipf 1.0 R / uniform S, 0.01-1 x "
                        "(200M + 50M) keys, rate 1 or 0.05), one batched launch of the persistent scan and join "
                        "kernels running concurrently%s"
                        % ("" if args.scale == 1.0 else " (scale %g)" % args.scale),
            "requests": len(reqs),
            "resident_bytes": resident,
            "sampled_rows": sel_rows,
            "join_keys_sampled": join_keys,
            "rows_predicates_per_step": rows_preds,
        },
        "schedule": sched,
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "kernel": dominant,
            "alg_bytes_per_launch": dk["alg_bytes"],
            "kernel_ms": round(dk["ms"], 4),
        },
        "kernels": {k: dict({"ms": round(v["ms"], 4), "alg_bytes": v["alg_bytes"],
                             "achieved_gbps": round(v["achieved_gbps"], 1),
                             "traffic": stored_traffic(k)}, **({"kernels": v["kernels"]} if "kernels" in v else {}))
                    for k, v in per_kernel.items()},
        "batch_kernel_span_ms": round(kernel_ms, 4),
        "host_compile_ms": round(compile_ms, 4),
        "graph_replay_ms_per_step": round(graph_ms, 4),
        "join_keys_per_s": join_keys / (wall / args.steps),
        "served": served,
        "plain_path": plain,
        "gate": gate,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
