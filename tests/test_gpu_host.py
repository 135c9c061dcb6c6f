"""Probes of host-resident tables (sampler on the device, gathered kept rows
copied to the device in chunks): every count equals the oracle's on the same
host arrays and the device-resident probe's, in both transfer modes, over
ragged chunks, row sampling, empty samples and a table with no rows."""
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
    w = datagen.config2(n_rows=1_000_003, rate=0.2)
    t = w.tables[0]
    host = datagen.host_table(t)
    ctx = g.gace_create(0, 2 << 30)
    yield g, w, t, host, ctx
    g.gace_destroy(ctx)


@pytest.mark.parametrize("rate,B,chunk,key_only", [(1.0, 4096, 0, True), (1.0, 4096, 0, False),
                                                   (0.2, 512, 4096, True), (0.2, 512, 70_000, False),
                                                   (0.05, 1, 65536, True), (0.0, 4096, 0, True),
                                                   (0.7, 1 << 20, 300_000, True)])
def test_host_probe_matches_oracle(env, rate, B, chunk, key_only):
    g, w, t, host, ctx = env
    preds = w.sel[0].preds[:24]
    dtypes = [c.dtype for c in t.cols]
    print("host probe", rate, B, chunk, key_only, flush=True)
    got = g.gace_probe_selectivity_host(ctx, host, t.table_id, preds, 31, rate, B, key_only=key_only,
                                        chunk_rows=chunk)
    want = oracle.probe_selectivity(host, dtypes, t.table_id, preds, 31, rate, B)
    assert got[0].tolist() == want[0].tolist() and got[1:3] == want[1:]
    st = got[3]
    used = sorted({c for p in preds for c, _, _ in p}) if key_only else list(range(len(host)))
    row_bytes = sum(host[c].dtype.itemsize for c in used)
    assert st["h2d_bytes"] == got[1] * row_bytes
    per = chunk or (1 << 22)
    assert st["chunks"] == (got[1] + per - 1) // per


def test_host_probe_equals_device_probe(env):
    import torch
    g, w, t, host, ctx = env
    preds = w.sel[0].preds
    dev = [torch.from_numpy(c).cuda() for c in host]
    for seed in (1, 2):
        a = g.gace_probe_selectivity_host(ctx, host, t.table_id, preds, seed, 0.3, 2048, chunk_rows=100_000)
        b = g.gace_probe_selectivity(ctx, g.Table(dev, t.table_id), preds, seed, 0.3, 2048)
        assert a[0].tolist() == b[0].tolist() and a[1:3] == b[1:]


def test_host_probe_edge_tables(env):
    g, w, t, host, ctx = env
    empty = [np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.int64)]
    c, n, k, st = g.gace_probe_selectivity_host(ctx, empty, 9, [[(0, g.EQ, (0,))], [(1, g.RANGE, (0, 5))]])
    assert c.tolist() == [0, 0] and (n, k) == (0, 0) and st["chunks"] == 0
    # one ragged block of 5 rows; no predicates at all
    small = [np.array([1, 2, 3, 2, 1], dtype=np.int32)]
    c, n, k, _ = g.gace_probe_selectivity_host(ctx, small, 9, [[(0, g.EQ, (2,))]])
    assert c.tolist() == [2] and (n, k) == (5, 1)
    c, n, k, st = g.gace_probe_selectivity_host(ctx, small, 9, [])
    assert (n, k) == (5, 1) and st["h2d_bytes"] == 0
    with pytest.raises(g.GaceError):
        g.gace_probe_selectivity_host(ctx, small, 9, [[(0, g.EQ, (2,))]], chunk_rows=100)
