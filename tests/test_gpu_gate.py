"""The gate's device-backed calls on the GPU: the one-probe PCS counts
{A, B, A AND B} and the cached probes equal the oracle's counts bit for bit,
and the gate's decisions on them equal the oracle's."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import gate as og

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2512_19750_amd as g
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = datagen.config2(n_rows=1_000_003, rate=0.2)
    t = w.tables[0]
    cols = datagen.device_table(t, dev)
    host = [c.cpu().numpy() for c in cols]
    ctx = g.gace_create(0, 2 << 30)
    yield g, w, t, cols, host, ctx
    g.gace_destroy(ctx)


def test_pcs_probe_matches_oracle(env):
    g, w, t, cols, host, ctx = env
    table = g.Table(cols, t.table_id)
    dtypes = [c.dtype for c in t.cols]
    preds = w.sel[0].preds
    pairs = [(preds[i], preds[i + 1]) for i in range(0, 24, 2) if len(preds[i]) + len(preds[i + 1]) <= 16]
    # c1 = c0 + U{-50..50}: strongly correlated; c3 is independent of c0
    a0 = [(0, g.RANGE, (1000, 1100))]
    pairs += [(a0, [(1, g.RANGE, (1000, 1100))]), (a0, [(1, g.RANGE, (5000, 100_000))]),
              (a0, [(3, g.RANGE, (0, 500_000))])]
    flags = []
    for a, b in pairs:
        print("pcs pair", a, b, flush=True)
        got = g.gace_probe_pcs(ctx, table, a, b, seed=5, rate=0.2, block_rows=512)
        want, n, _ = oracle.probe_selectivity(host, dtypes, t.table_id, [a, b, a + b], 5, 0.2, 512)
        assert (got.c_a, got.c_b, got.c_ab, got.n_pcs) == (int(want[0]), int(want[1]), int(want[2]), n)
        d = g.gace_gate_evaluate(pcs=got)
        o = og.gate(pcs=(int(want[2]), int(want[0]), int(want[1]), n))
        assert d["flags"] == o["flags"] and d["undefined"] == o["undefined"]
        flags.append(o["flags"])
    assert flags[-3] == og.PCS_HI and flags[-2] == og.PCS_LO and flags[-1] == 0


def test_cached_probe_equals_oracle(env):
    g, w, t, cols, host, ctx = env
    table = g.Table(cols, t.table_id)
    dtypes = [c.dtype for c in t.cols]
    preds = w.sel[0].preds
    c = g.gace_cache_create(1000)
    try:
        def check(ps, n_hit):
            got = g.gace_probe_selectivity_cached(ctx, c, table, ps, 9, 0.2, 512)
            want = oracle.probe_selectivity(host, dtypes, t.table_id, ps, 9, 0.2, 512)
            assert got[0].tolist() == want[0].tolist() and got[1:3] == want[1:]
            assert got[3] == n_hit
        check(preds[:20], 0)
        check(preds[:20], 20)
        check(preds[10:30], 10)            # half cached: only the rest is probed
        check(preds[5:6], 1)
        g.gace_cache_invalidate(c, t.table_id)
        check(preds[:20], 0)
        st = g.gace_cache_stats_get(c)
        assert st["entries"] == 20 and st["invalidated"] == 30   # 30 dropped, 20 probed again
    finally:
        g.gace_cache_destroy(c)


def test_cached_join_equals_oracle(env):
    g, w, t, cols, host, ctx = env
    r, s = datagen.join_pair(300_000, 100_000, 50_000, 77, 5, 6)
    import torch
    kr = datagen.device_column(r.cols[0], r.n_rows, torch.device("cuda:0"))
    ks = datagen.device_column(s.cols[0], s.n_rows, torch.device("cuda:0"))
    c = g.gace_cache_create(8)
    try:
        R, S = g.Keys(kr, 5, 1, 0.5, 256), g.Keys(ks, 6, 2, 0.5, 256)
        want = oracle.join_freq(kr.cpu().numpy(), 5, 1, 0.5, 256, ks.cpu().numpy(), 6, 2, 0.5, 256)
        got, hit = g.gace_join_freq_cached(ctx, c, R, S)
        assert got == want and not hit
        got, hit = g.gace_join_freq_cached(ctx, c, R, S)
        assert got == want and hit
        g.gace_cache_invalidate(c, 6)
        got, hit = g.gace_join_freq_cached(ctx, c, R, S)
        assert got == want and not hit
    finally:
        g.gace_cache_destroy(c)
