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
JOIN_FIELDS = ["join_card", "ndv_R", "ndv_S", "n_R", "n_S", "f1_R", "f1_S", "f2_R", "f2_S"]
CSRC = os.path.join(ROOT, "paper_2512_19750_amd", "csrc")
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("kernels.hip", "plan.h", "compile.cpp")]


def kernel_hash() -> str:
    """Hash of the sources that decide what the kernels read and write."""
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counters_path(kernel: str, workload: str = "c4") -> str:
    return os.path.join(ROOT, "profiles", "%s_%s_counters.md" % (kernel, workload))


def stored_counters(kernel: str, workload: str = "c4") -> dict:
    """Figures per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (`name: value` lines), if it was taken on the
    current kernel sources (else {})."""
    path = counters_path(kernel, workload)
    if not os.path.exists(path):
        return {}
    out = {}
    for line in open(path).read().splitlines():
        if ":" not in line or line.startswith(("|", "#", " ")):
            continue
        k, v = line.split(":", 1)
        try:
            out[k.strip()] = float(v.strip())
        except ValueError:
            out[k.strip()] = v.strip()
    if out.get("kernel_source_sha256_16") != kernel_hash():
        return {}
    return out


def stored_traffic(kernel: str, workload: str = "c4"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None)."""
    return stored_counters(kernel, workload).get("hbm_bytes_per_launch")


def read_ceiling(g, dev, n_bytes: int = 4 << 30, reps: int = 10) -> dict:
    """HBM read ceiling of this GPU: the read kernel over a zero-filled
    n_bytes buffer, median device time of `reps` runs after two warm-ups."""
    import torch
    buf = torch.zeros(n_bytes // 4, dtype=torch.int32, device=dev)
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    for _ in range(2):
        g.gace_read_ceiling(buf, sink)
    ms = sorted(g.gace_read_ceiling(buf, sink) for _ in range(reps))
    del buf
    torch.cuda.empty_cache()
    med = ms[len(ms) // 2]
    return dict(gbps=round(n_bytes / (med * 1e-3) / 1e9, 1), best_gbps=round(n_bytes / (ms[0] * 1e-3) / 1e9, 1),
                bytes=n_bytes, reps=reps, kernel="gace_read_kernel")


def cpu_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(cpu_model=model, host_logical_cpus=os.cpu_count())


# the oracle's threads: the host cores allotted to one GPU (at most 16)
CPU_THREADS = min(os.cpu_count() or 1, 16)


def stored_expected(name: str, w):
    """The oracle's stored results for workload `name` (c4 or c5), in the
    workload's request order, as the tuples the comparisons use; None when the
    stored file was written for another workload definition (a scaled run)."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import expected_io
    try:
        d = expected_io.load(name, w)
    except ValueError:
        return None
    out = []
    for kind, i in w.order:
        v = d[(kind, i)]
        if kind == "join":
            out.append(tuple(v[f] for f in expected_io.JOIN_FIELDS))
        else:
            out.append((tuple(v[0]), v[1], v[2]))
    return out


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


def cpu_baseline(w, budget_rows_preds: float, nthreads: int, join_keys_budget: float = 3e7):
    """The oracle on bounded samples of the batch: selectivity requests taken
    in batch order until the sample holds ~budget rows*predicates, counted on
    `nthreads` threads and (a share of them) on one thread; and join requests
    in batch order until ~join_keys_budget sampled keys, joined by the
    oracle's sort (one thread)."""
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
    secs1, rp1, n1 = 0.0, 0, 0
    for i, kb in picked:
        r = w.sel[i]
        t = w.tables[r.table]
        spans = oracle.merge_spans([(int(b) * r.spec.block_rows, min(t.n_rows, (int(b) + 1) * r.spec.block_rows))
                                    for b in kb])
        cols = [np.concatenate([datagen.host_column(c, e - b, row0=b, nthreads=nthreads) for b, e in spans])
                for c in t.cols]
        dts = [c.dtype for c in t.cols]
        t0 = time.perf_counter()
        counts, sampled, _ = oracle.probe_selectivity(cols, dts, t.table_id, r.preds, 0, 1.0, 1 << 20, nthreads)
        secs += time.perf_counter() - t0
        rp_done += sampled * len(r.preds)
        rows_done += sampled
        if rp1 + sampled * len(r.preds) <= budget_rows_preds / nthreads:
            t0 = time.perf_counter()
            c1, _, _ = oracle.probe_selectivity(cols, dts, t.table_id, r.preds, 0, 1.0, 1 << 20, 1)
            secs1 += time.perf_counter() - t0
            assert c1.tolist() == counts.tolist()
            rp1 += sampled * len(r.preds)
            n1 += 1
        del cols
    # joins: the oracle's sort-based frequency join on the regenerated kept keys
    jsecs, jkeys, jn = 0.0, 0, 0
    for kind, j in w.order:
        if kind != "join":
            continue
        jr = w.joins[j]
        est = 0
        for side, sp in ((jr.r, jr.spec_r), (jr.s, jr.spec_s)):
            kb = oracle.kept_blocks(side.n_rows, sp.seed, side.table_id, sp.rate, sp.block_rows)
            est += len(kb) * sp.block_rows
        if est == 0 or jkeys + est > join_keys_budget:
            continue
        kr = oracle.sampled_keys(jr.r, jr.spec_r, nthreads)
        ks = oracle.sampled_keys(jr.s, jr.spec_s, nthreads)
        t0 = time.perf_counter()
        oracle.join_freq(kr, jr.r.table_id, 0, 1.0, 1 << 20, ks, jr.s.table_id, 0, 1.0, 1 << 20)
        jsecs += time.perf_counter() - t0
        jkeys += len(kr) + len(ks)
        jn += 1
        del kr, ks
    out = dict(value=rp_done / secs if secs > 0 else None, unit="rows*predicates/s", cores=nthreads,
               kind="oracle", seconds=round(secs, 3),
               sample="%d of %d selectivity requests in batch order (%d sampled rows, %.3g rows*predicates); "
                      "kept-block rows regenerated on the host, counting timed"
                      % (len(picked), len(w.sel), rows_done, rp_done),
               t1=dict(value=rp1 / secs1 if secs1 > 0 else None, unit="rows*predicates/s", cores=1,
                       seconds=round(secs1, 3),
                       sample="the first %d of those requests (%.3g rows*predicates), same counts" % (n1, rp1)),
               join=dict(value=jkeys / jsecs if jsecs > 0 else None, unit="sampled join keys/s", cores=1,
                         seconds=round(jsecs, 3),
                         sample="%d of %d join requests in batch order (%d sampled keys, R + S), sort-based "
                                "frequency join timed" % (jn, len(w.joins), jkeys)))
    out.update(cpu_info())
    return out


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
    with the pool entry's expected result (the oracle's stored one at full
    size)."""
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
                got = tuple(int(getattr(o, f)) for f in JOIN_FIELDS)
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
                completed_early=stats["completed_early"], workspace_peak=stats["workspace_peak"])


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
            expect.append(tuple(r[f] for f in JOIN_FIELDS))
        else:
            c, nrow, nblk = g.gace_probe_selectivity(ctx, q.table, q.preds, q.seed, q.rate, q.block_rows)
            expect.append((tuple(int(x) for x in c), nrow, nblk))
        plain_lat.append((time.perf_counter() - s0) * 1e3)
    g.gace_destroy(ctx)
    plain_s = time.time() - t0
    print("[serve] plain path over the pool: %.1fs (%.1f req/s)" % (plain_s, len(pool) / plain_s), file=sys.stderr,
          flush=True)
    # served results are compared with the oracle's stored pool results (at
    # full size), which the plain path must equal too
    oracle_expect = stored_expected("c5", w)
    plain_vs_oracle = None
    if oracle_expect is not None:
        plain_vs_oracle = sum(a != b for a, b in zip(expect, oracle_expect))
        expect = oracle_expect
    reference = "oracle (stored pool results)" if oracle_expect is not None else "plain path (scaled run)"
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
        "served_results_compared_with": reference,
        "plain_path_pool": {"seconds": round(plain_s, 3), "mismatches_vs_oracle": plain_vs_oracle,
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


# ---------------------------------------------------------------- configs 1-3
def _lat(xs):
    return dict(p50=round(_pct(xs, 0.50), 3), p99=round(_pct(xs, 0.99), 3), min=round(min(xs), 3))


def _sel_cpu(cols_host, dtypes, table_id, preds, seed, rate, B, want, min_s=2.0):
    """The oracle on the same probe: per-probe seconds on CPU_THREADS threads
    and on one, each repeated until min_s has passed; its counts must equal
    `want` (the device's)."""
    import oracle
    res = {}
    for T in (CPU_THREADS, 1):
        n, t_all = 0, 0.0
        while t_all < min_s or n < 1:
            t0 = time.perf_counter()
            got = oracle.probe_selectivity(cols_host, dtypes, table_id, preds, seed, rate, B, T)
            t_all += time.perf_counter() - t0
            n += 1
        if got[0].tolist() != want[0].tolist() or got[1] != want[1]:
            raise RuntimeError("device counts differ from the oracle's")
        res[T] = (t_all / n, n)
    return res


def config_sel_main(args, cfg: int):
    """Configs 1 and 2: one selectivity probe on the plain path (call to
    results on the host), repeated; latency percentiles, device time of the
    scan kernel from its HIP events, and the same probe on the allocation-free
    entry point."""
    import torch

    import datagen
    import paper_2512_19750_amd as g
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ceiling = read_ceiling(g, dev)
    w = datagen.config1() if cfg == 1 else datagen.config2()
    t = w.tables[0]
    req = w.sel[0]
    sp = req.spec
    t_setup = time.time()
    cols = datagen.device_table(t, dev)
    torch.cuda.synchronize()
    print("[bench] config %d: %d rows x %d columns generated in %.1fs" % (cfg, t.n_rows, len(t.cols),
                                                                         time.time() - t_setup),
          file=sys.stderr, flush=True)
    tab = g.Table(cols, t.table_id)
    ctx = g.gace_create(0, 1 << 30)
    reps = args.reps or (2000 if cfg == 1 else 300)
    # marshalled once: each timed call is one C ABI call (compile, upload,
    # kernels, download, sync)
    probe = g.PreparedProbe(tab, req.preds, sp.seed, sp.rate, sp.block_rows)
    for _ in range(args.warmup * 10):
        probe.run(ctx)
    lat, kern = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        probe.run(ctx)
        lat.append((time.perf_counter() - t0) * 1e6)
        ks = g.gace_last_kernel_stats(ctx)
        kern.append(ks["scan_ms"] * 1e3)
    got = probe.run(ctx)
    got = (got[0].copy(), got[1], got[2])
    alg = ks["scan_alg_bytes"]
    compile_us = ks["compile_ms"] * 1e3
    g.gace_destroy(ctx)
    # the entry point's first call on a device looks up its scratch: warm up
    # as the context path does
    for _ in range(args.warmup * 10):
        probe.run_noalloc()
    na = []
    for _ in range(reps):
        t0 = time.perf_counter()
        got_na = probe.run_noalloc()
        na.append((time.perf_counter() - t0) * 1e6)
    if got_na[0].tolist() != got[0].tolist() or got_na[1:] != got[1:]:
        raise RuntimeError("allocation-free probe differs from the context path")
    sampled, n_preds = got[1], len(req.preds)
    k_mean = sum(kern) / len(kern)
    achieved = alg / (k_mean * 1e-6) / 1e9
    p50 = _pct(lat, 0.5)
    cpu = None
    if not args.no_cpu:
        host = [c.cpu().numpy() for c in cols]
        if cfg == 2:        # the kept blocks only (1 % of the rows), regenerated as the oracle does
            import oracle
            kb = oracle.kept_blocks(t.n_rows, sp.seed, t.table_id, sp.rate, sp.block_rows)
            rows = np.concatenate([np.arange(int(b) * sp.block_rows, min(t.n_rows, (int(b) + 1) * sp.block_rows))
                                   for b in kb]) if len(kb) else np.zeros(0, dtype=np.int64)
            host = [h[rows] for h in host]
            seed, rate, B = 0, 1.0, 1 << 20
            sample = "the probe's %d kept blocks (%d rows), counted on the host" % (len(kb), len(rows))
        else:
            seed, rate, B = sp.seed, sp.rate, sp.block_rows
            sample = "the whole probe (%d rows)" % t.n_rows
        r = _sel_cpu(host, [c.dtype for c in t.cols], t.table_id, req.preds, seed, rate, B, got)
        cpu = dict(value=r[CPU_THREADS][0] * 1e6, unit="us per probe", cores=CPU_THREADS, kind="oracle",
                   sample=sample + ", repeated %d times; counts equal the device's" % r[CPU_THREADS][1],
                   t1=dict(value=r[1][0] * 1e6, unit="us per probe", cores=1, repeats=r[1][1]),
                   rows_predicates_per_s=sampled * n_preds / r[CPU_THREADS][0])
        cpu.update(cpu_info())
    sq = stored_counters("gace_scan_kernel", "c%d" % cfg)
    valu = sq.get("sq_insts_valu_per_launch")
    salu = sq.get("sq_insts_salu_per_launch")
    out = {
        "metric": "plain single-probe latency (call to counts on the host), p50",
        "value": round(p50, 3),
        "unit": "us",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup * 10,
        "ms_per_step": round(p50 / 1e3, 6),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if cfg == 1 else "int32,int64,f32",
        "data": "synthetic (seeded counter-based generator, generated in HBM)",
        "config": {"workload": ("C1 plain single probe: 1,000,000 rows x 4 int32 U[0,1000), c0 in [100,300) AND "
                                "c1 in [0,500), rate 1" if cfg == 1 else
                                "C2 skewed correlated multi-predicate probe: 100M rows x 8 columns (Zipf 1.1, "
                                "Zipf 1.1 + noise, Zipf 1.3, uniform i32, 2 uniform i64, 2 uniform f32), 64 "
                                "predicates of 2-4 terms, block-Bernoulli 1 %, 4096-row blocks"),
                   "sampled_rows": sampled, "kept_blocks": got[2], "predicates": n_preds},
        "latency_us": _lat(lat),
        "scan_kernel_us": _lat(kern),
        "host_compile_us": round(compile_us, 3),
        "noalloc_latency_us": _lat(na),
        "rows_predicates_per_s": sampled * n_preds / (p50 * 1e-6),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": stored_traffic("gace_scan_kernel", "c%d" % cfg), "kernel": "gace_scan_kernel",
                     "alg_bytes_per_launch": alg, "kernel_us": round(k_mean, 3),
                     "read_ceiling_gbps": ceiling["gbps"]},
        "issue_counts": None if valu is None else {
            "kernel": "gace_scan_kernel", "sq_insts_valu_per_launch": valu, "sq_insts_salu_per_launch": salu,
            "valu_lane_ops_per_sampled_row": round(valu * 64 / max(sampled, 1), 2),
            "valu_lane_ops_per_alg_byte": round(valu * 64 / max(alg, 1), 3)},
        "read_ceiling": ceiling,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def config3_main(args):
    """Config 3: the join-key frequency probe on the plain path at 100 % and
    5 % sampling; keys/s of the call, and the join stage's device time from its
    HIP events against its algorithmic bytes."""
    import torch

    import datagen
    import paper_2512_19750_amd as g
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ceiling = read_ceiling(g, dev)
    w1 = datagen.config3(1.0)
    jr = w1.joins[0]
    t_setup = time.time()
    kr = datagen.device_column(jr.r.cols[0], jr.r.n_rows, dev)
    ks = datagen.device_column(jr.s.cols[0], jr.s.n_rows, dev)
    torch.cuda.synchronize()
    print("[bench] config 3: %d + %d keys generated in %.1fs" % (jr.r.n_rows, jr.s.n_rows, time.time() - t_setup),
          file=sys.stderr, flush=True)
    ctx = g.gace_create(0, 24 << 30)
    lines = []
    for rate in (1.0, 0.05):
        w = datagen.config3(rate)
        j = w.joins[0]
        R = g.Keys(kr, j.r.table_id, j.spec_r.seed, rate, j.spec_r.block_rows)
        S = g.Keys(ks, j.s.table_id, j.spec_s.seed, rate, j.spec_s.block_rows)
        steps = args.steps if rate == 1.0 else args.steps * 5
        for _ in range(args.warmup):
            res = g.gace_join_freq(ctx, R, S)
        torch.cuda.synchronize()
        wall, dev_ms = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            res = g.gace_join_freq(ctx, R, S)
            wall.append((time.perf_counter() - t0) * 1e3)
            st = g.gace_last_kernel_stats(ctx)
            dev_ms.append(st["join_ms"])
        keys = res["n_R"] + res["n_S"]
        alg = st["join_alg_bytes"]
        jm = sum(dev_ms) / len(dev_ms)
        wm = _pct(wall, 0.5)
        achieved = alg / (jm * 1e-3) / 1e9
        tag = "c3r%d" % round(rate * 100)
        traffic = stored_traffic("gace_join_stage", tag)
        cpu = None
        if not args.no_cpu and rate == 0.05:
            import oracle
            r_keys = oracle.sampled_keys(j.r, j.spec_r, CPU_THREADS)
            s_keys = oracle.sampled_keys(j.s, j.spec_s, CPU_THREADS)
            t0 = time.perf_counter()
            want = oracle.join_freq(r_keys, j.r.table_id, 0, 1.0, 1 << 20, s_keys, j.s.table_id, 0, 1.0, 1 << 20)
            secs = time.perf_counter() - t0
            if want != res:
                raise RuntimeError("device join result differs from the oracle's")
            cpu = dict(value=(len(r_keys) + len(s_keys)) / secs, unit="sampled keys/s", cores=1, kind="oracle",
                       seconds=round(secs, 3),
                       sample="the 5 %% probe's %d kept keys (R + S), sort-based frequency join; result equals "
                              "the device's" % (len(r_keys) + len(s_keys)))
            cpu.update(cpu_info())
        lines.append({
            "metric": "join-key frequency probe: sampled keys/s (call to results on the host)",
            "value": keys / (wm * 1e-3),
            "unit": "keys/s",
            "n_gpus": 1,
            "steps": steps,
            "warmup": args.warmup,
            "ms_per_step": round(wm, 4),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "int64",
            "data": "synthetic (seeded counter-based generator, generated in HBM)",
            "config": {"workload": "C3 join-key frequency probe: R 200M int64 Zipf 1.0 over 1e7 keys, S 50M "
                                   "uniform over the same domain, rate %g, 4096-row blocks" % rate,
                       "sampled_keys": keys, "ndv_R": res["ndv_R"], "ndv_S": res["ndv_S"],
                       "join_card": res["join_card"]},
            "wall_ms": _lat(wall),
            "join_stage_ms": round(jm, 4),
            "device_keys_per_s": keys / (jm * 1e-3),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                         "traffic_gbps": None if traffic is None else round(traffic / (jm * 1e-3) / 1e9, 1),
                         "kernel": "gace_join_stage", "alg_bytes_per_launch": alg, "kernel_ms": round(jm, 4),
                         "read_ceiling_gbps": ceiling["gbps"]},
            "read_ceiling": ceiling,
            "cpu_baseline": cpu,
        })
        print("[bench] config 3 rate %g: %.3f ms wall, %.3f ms join stage, %.3g keys/s"
              % (rate, wm, jm, keys / (wm * 1e-3)), file=sys.stderr, flush=True)
    g.gace_destroy(ctx)
    for line in lines:
        print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--config", type=int, default=4, choices=[1, 2, 3, 4],
                    help="1/2: plain single-probe latency; 3: join probe at 100 %% and 5 %%; 4: the batch")
    ap.add_argument("--reps", type=int, default=0, help="probes timed in --config 1/2 (0: 2000 / 300)")
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
        print("bench.py measures one GPU: the library runs the probe on a single MI355X "
              "(sharding across GPUs is described, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.config in (1, 2):
        config_sel_main(args, args.config)
        return
    if args.config == 3:
        config3_main(args)
        return
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
    ceiling = read_ceiling(g, dev)
    print("[bench] HBM read ceiling %.0f GB/s (best %.0f)" % (ceiling["gbps"], ceiling["best_gbps"]),
          file=sys.stderr, flush=True)
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
    # the timed region replays the captured graph (the batched path's launch),
    # so the schedule is tuned in that launch mode; the graph holds HIP timing
    # events around the scan kernel (call's stream) and the join stage (side
    # stream), read after every step
    g.gace_set_graph(ctx, True)
    if args.autotune:
        t0 = time.time()
        g.gace_autotune(ctx, reqs, args.tune_cache)
        print("[bench] schedule %s (%.1fs)" % (g.gace_get_schedule(ctx), time.time() - t0), file=sys.stderr,
              flush=True)
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
    if not ks["timed"] or min(sms) <= 0 or min(jms) <= 0:
        raise RuntimeError("the graph replay returned no per-kernel times")
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
    # direct launches of the same batch (the plain path's launch mode), for comparison
    g.gace_set_graph(ctx, False)
    g.gace_batch_run(ctx, reqs, prepared=prepared)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.gace_batch_run(ctx, reqs, prepared=prepared)
    torch.cuda.synchronize()
    direct_ms = (time.perf_counter() - t0) / args.steps * 1e3
    g.gace_set_graph(ctx, True)
    sel_rows = 0
    join_keys = 0
    for q in reqs:
        if isinstance(q, g.JoinRequest):
            r = q.result()
            join_keys += r["n_R"] + r["n_S"]
        else:
            sel_rows += q.result()[1]
    compile_ms = sum(cms) / len(cms)
    print("[bench] batch %.2f ms/step graph replay (host compile %.2f ms, kernels %.2f ms: scan %.2f, join %.2f; "
          "direct launch %.2f ms/step), %.3g rows*preds/s"
          % (ms_step, compile_ms, kernel_ms, per_kernel["gace_scan_kernel"]["ms"],
             per_kernel["gace_join_stage"]["ms"], direct_ms, value), file=sys.stderr, flush=True)

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
                expect.append(tuple(r[f] for f in JOIN_FIELDS))
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
    # served: the same requests arriving as an open-loop Poisson stream; each
    # result is compared with the oracle's stored result (full size)
    served = None
    if args.plain and args.serve_point_qps > 0:
        kinds = ["join" if isinstance(q, g.JoinRequest) else "sel" for q in reqs]
        oracle_expect = stored_expected("c4", w)
        ref = expect if oracle_expect is None else oracle_expect
        served = serve_point(g, prepared[0], ref, kinds, args.serve_point_qps,
                             dict(max_inflight=3, max_batch=64, queue_capacity=4096, workspace_bytes=ws),
                             seed=S_SERVE, duration_s=args.serve_point_seconds)
        served["compared_with"] = "plain path (scaled run)" if oracle_expect is None else "oracle (stored results)"
        if oracle_expect is not None:
            served["plain_mismatches_vs_oracle"] = sum(a != b for a, b in zip(expect, oracle_expect))
        print("[bench] served %s" % json.dumps(served), file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_budget * args.scale, CPU_THREADS)
        print("[bench] oracle %.3g rows*preds/s on %d threads (%.1fs), %.3g on 1 (%.1fs); join %.3g keys/s"
              % (cpu["value"] or 0, CPU_THREADS, cpu["seconds"], cpu["t1"]["value"] or 0, cpu["t1"]["seconds"],
                 cpu["join"]["value"] or 0), file=sys.stderr, flush=True)

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
                        "(200M + 50M) keys, rate 1 or 0.05), one graph-replayed launch of the persistent scan "
                        "and join kernels running concurrently%s"
                        % ("" if args.scale == 1.0 else " (scale %g)" % args.scale),
            "requests": len(reqs),
            "resident_bytes": resident,
            "sampled_rows": sel_rows,
            "join_keys_sampled": join_keys,
            "rows_predicates_per_step": rows_preds,
            "launch": "hipGraph replay",
        },
        "schedule": sched,
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            # HBM bytes the counters saw per launch, over the same event time
            "traffic_gbps": None if traffic is None else round(traffic / (dk["ms"] * 1e-3) / 1e9, 1),
            "traffic_frac": None if traffic is None else round(traffic / (dk["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "kernel": dominant,
            "alg_bytes_per_launch": dk["alg_bytes"],
            "kernel_ms": round(dk["ms"], 4),
            "read_ceiling_gbps": ceiling["gbps"],
            "frac_of_read_ceiling": round(achieved / ceiling["gbps"], 4),
        },
        "kernels": {k: dict({"ms": round(v["ms"], 4), "alg_bytes": v["alg_bytes"],
                             "achieved_gbps": round(v["achieved_gbps"], 1),
                             "traffic": stored_traffic(k),
                             "traffic_gbps": (None if stored_traffic(k) is None or not v["ms"] else
                                              round(stored_traffic(k) / (v["ms"] * 1e-3) / 1e9, 1))},
                            **({"kernels": v["kernels"]} if "kernels" in v else {}))
                    for k, v in per_kernel.items()},
        "read_ceiling": ceiling,
        "batch_kernel_span_ms": round(kernel_ms, 4),
        "host_compile_ms": round(compile_ms, 4),
        "direct_launch_ms_per_step": round(direct_ms, 4),
        "join_keys_per_s": join_keys / (wall / args.steps),
        "served": served,
        "plain_path": plain,
        "gate": gate,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
