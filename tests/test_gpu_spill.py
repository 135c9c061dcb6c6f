"""Sparse selectivity scans in small batches: an item scans the first kept
block of its 64-block sampling chunk and spills the chunk's other kept blocks
to a list that idle workgroups run.  Every count and sampled-row figure
equals the oracle's, with several kept blocks per chunk (rates up to 1/8),
ragged last blocks, more than one predicate group, zone maps, a batch that
also holds a join (per-request completion), and the allocation-free entry
point."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

INT32_MIN, INT32_MAX = -(2**31), 2**31 - 1


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2512_19750_amd as g
    torch.cuda.set_device(0)
    ctx = g.gace_create(0, 2 << 30)
    yield g, ctx, torch.device("cuda:0")
    g.gace_destroy(ctx)


def _table(rng, n):
    c0 = rng.integers(-1000, 1000, n).astype(np.int32)
    c1 = np.sort(rng.integers(0, 1_000_000, n)).astype(np.int32)       # clustered: zone maps can prune
    c2 = rng.integers(-(2**40), 2**40, n).astype(np.int64)
    c3 = rng.random(n).astype(np.float32)
    return [c0, c1, c2, c3], [1, 1, 2, 3]


def _preds(rng, n_preds):
    from paper_2512_19750_amd import RANGE
    out = []
    for p in range(n_preds):
        lo = int(rng.integers(-1000, 900))
        terms = [(0, RANGE, (lo, lo + int(rng.integers(1, 400))))]       # on c0
        if p % 3 == 1:
            a = int(rng.integers(0, 990_000))
            terms.append((1, RANGE, (a, a + 5000)))                      # narrow range on the sorted column
        if p % 3 == 2:
            terms.append((3, RANGE, (0.0, float(rng.random()))))
        out.append(terms)
    return out


@pytest.mark.parametrize("n,B,rate,n_preds", [(3_000_001, 4096, 0.12, 5), (2_000_000, 1024, 0.05, 70),
                                               (900_000, 512, 0.01, 3), (5_000_000, 4096, 0.002, 130)])
def test_sparse_probe_vs_oracle(env, n, B, rate, n_preds):
    import torch
    g, ctx, dev = env
    rng = np.random.default_rng(n + B)
    host, dtypes = _table(rng, n)
    preds = _preds(rng, n_preds)
    _say("sparse probe", n, B, rate, n_preds)
    table = g.Table([torch.from_numpy(c).to(dev) for c in host], 71)
    got = g.gace_probe_selectivity(ctx, table, preds, seed=9, rate=rate, block_rows=B)
    want = oracle.probe_selectivity(host, dtypes, 71, preds, 9, rate, B)
    assert got[0].tolist() == want[0].tolist() and got[1:] == want[1:]
    na = g.gace_probe_selectivity_noalloc(table, preds, seed=9, rate=rate, block_rows=B)
    assert na[0].tolist() == want[0].tolist() and na[1:] == want[1:]


def test_sparse_probe_with_zone_map(env):
    import torch
    g, ctx, dev = env
    rng = np.random.default_rng(5)
    host, dtypes = _table(rng, 4_000_000)
    preds = [[(1, g.RANGE, (100_000, 130_000))], [(1, g.RANGE, (500_000, 501_000)), (0, g.RANGE, (-10, 10))]]
    table = g.Table([torch.from_numpy(c).to(dev) for c in host], 72)
    zm = g.gace_zonemap_build(ctx, table)
    try:
        g.gace_zonemap_attach(ctx, zm)
        got = g.gace_probe_selectivity(ctx, table, preds, seed=4, rate=0.1, block_rows=4096)
        g.gace_zonemap_detach(ctx, zm)
    finally:
        g.gace_zonemap_destroy(zm)
    want = oracle.probe_selectivity(host, dtypes, 72, preds, 4, 0.1, 4096)
    assert got[0].tolist() == want[0].tolist() and got[1:] == want[1:]


def test_sparse_probes_in_a_batch_with_a_join(env):
    """Several sparse probes (one spilling, one dense) and a join in one
    batch: per-request completion publishes the counters after the spilled
    blocks have run."""
    import torch
    g, ctx, dev = env
    rng = np.random.default_rng(11)
    host, dtypes = _table(rng, 2_500_000)
    host2, _ = _table(rng, 700_000)
    table = g.Table([torch.from_numpy(c).to(dev) for c in host], 73)
    table2 = g.Table([torch.from_numpy(c).to(dev) for c in host2], 74)   # a dense scan of its own
    pa, pb = _preds(rng, 9), _preds(rng, 4)
    r = rng.integers(0, 5000, 400_000).astype(np.int64)
    s = rng.integers(0, 5000, 100_000).astype(np.int64)
    kr, ks = torch.from_numpy(r).to(dev), torch.from_numpy(s).to(dev)
    reqs = [g.SelRequest(table, pa, seed=3, rate=0.08, block_rows=4096),
            g.SelRequest(table2, pb, seed=3, rate=0.9, block_rows=4096),
            g.JoinRequest(g.Keys(kr, 81, 1, 0.5, 4096), g.Keys(ks, 82, 2, 0.5, 4096))]
    g.gace_batch_run(ctx, reqs)
    for q, cols, tid, preds, rate in ((reqs[0], host, 73, pa, 0.08), (reqs[1], host2, 74, pb, 0.9)):
        c, n, b = q.result()
        want = oracle.probe_selectivity(cols, dtypes, tid, preds, 3, rate, 4096)
        assert c.tolist() == want[0].tolist() and (n, b) == want[1:]
    assert reqs[2].result() == oracle.join_freq(r, 81, 1, 0.5, 4096, s, 82, 2, 0.5, 4096)
