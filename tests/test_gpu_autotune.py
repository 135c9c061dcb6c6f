"""Autotuner on the GPU: it picks a valid schedule for a batch's shape, the
batch's results under the tuned schedule equal those under the default one,
and the schedule cache file written by one context is read back by the next
(same schedule, no new search)."""
import json
import os
import time

import pytest

import datagen

pytestmark = pytest.mark.gpu


def _requests(g, w, tabs, keys):
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


def _results(reqs):
    return [q.result() if hasattr(q, "R") else (q.result()[0].tolist(), q.result()[1], q.result()[2]) for q in reqs]


def test_autotune_picks_valid_schedule_and_caches_it(tmp_path):
    import torch

    import paper_2512_19750_amd as g
    torch.cuda.set_device(0)
    w = datagen.config4(scale=0.002, n_sel=40, n_join=6, seed_offset=23)
    tabs, keys = datagen.materialise(w, torch.device("cuda:0"))
    reqs = _requests(g, w, tabs, keys)
    cache = str(tmp_path / "tuned.jsonl")
    ctx = g.gace_create(0, 2 << 30)
    try:
        g.gace_batch_run(ctx, reqs)
        base = _results(reqs)
        g.gace_autotune(ctx, reqs, cache)
        s = g.gace_get_schedule(ctx)
        assert 1 <= s["wgs_per_cu"] <= 8 and 1 <= s["join_wgs_per_cu"] <= 4 and 1 <= s["agg_wgs_per_cu"] <= 8
        assert s["item_rows"] >= 1024 and s["count_mode"] in (0, 1, 2) and s["join_part_keys"] in (512, 1024, 2048)
        g.gace_batch_run(ctx, reqs)
        assert _results(reqs) == base
    finally:
        g.gace_destroy(ctx)
    lines = [json.loads(x) for x in open(cache).read().splitlines() if x.strip()]
    assert len(lines) == 1 and lines[0]["schedule"] == s
    ctx = g.gace_create(0, 2 << 30)
    try:
        t0 = time.perf_counter()
        g.gace_autotune(ctx, reqs, cache)          # a cache hit: no search
        assert time.perf_counter() - t0 < 0.5
        assert g.gace_get_schedule(ctx) == s
    finally:
        g.gace_destroy(ctx)
