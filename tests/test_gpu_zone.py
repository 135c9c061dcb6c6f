"""Zone maps on the GPU: the per-zone minima and maxima equal the oracle's,
the zones the prune pass skips are exactly the oracle's, and every count of a
zone-pruned probe equals the oracle's and the unpruned probe's, on clustered
and unclustered tables, sampled and full scans, blocks spanning many zones
and blocks inside one zone."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import zonemap as oz

pytestmark = pytest.mark.gpu

INT32_MIN, INT32_MAX = -(2**31), 2**31 - 1
INT64_MIN, INT64_MAX = -(2**63), 2**63 - 1


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2512_19750_amd as g
    torch.cuda.set_device(0)
    ctx = g.gace_create(0, 2 << 30)
    yield g, torch, ctx
    g.gace_destroy(ctx)


def _edge_table(n, rng):
    c0 = np.sort(rng.integers(0, 1_000_000, n)).astype(np.int32)           # clustered
    c1 = rng.integers(INT32_MIN, INT32_MAX, n, dtype=np.int64).astype(np.int32)
    c1[[0, 7, n - 1]] = [INT32_MIN, INT32_MAX, INT32_MIN]
    c2 = np.sort(rng.integers(-2**62, 2**62, n)).astype(np.int64)
    c2[[3, n - 2]] = [INT64_MIN, INT64_MAX]
    c3 = rng.random(n).astype(np.float32)
    c3[4096:8192] = np.nan                                                 # zone 1: NaN only
    c3[[10, 20_000]] = [np.float32(-0.0), np.float32(np.inf)]
    return [c0, c1, c2, c3], [1, 1, 2, 3]


def _check_zonemap(g, zm, host, dtypes):
    for c, (col, dt) in enumerate(zip(host, dtypes)):
        lo, hi = g.gace_zonemap_read(zm, c, col.dtype)
        wlo, whi = oz.zone_minmax(col)
        assert np.array_equal(lo, wlo) and np.array_equal(hi, whi), c


def test_zonemap_values_match_oracle(env):
    g, torch, ctx = env
    rng = np.random.default_rng(3)
    host, dtypes = _edge_table(100_000 + 333, rng)
    dev = [torch.from_numpy(c).cuda() for c in host]
    zm = g.gace_zonemap_build(ctx, g.Table(dev, 5))
    try:
        assert g.gace_zonemap_info(zm) == (host[0].size + 4095) // 4096
        _check_zonemap(g, zm, host, dtypes)
    finally:
        g.gace_zonemap_destroy(zm)


@pytest.mark.parametrize("rate,B", [(1.0, 4096), (0.3, 512), (0.5, 1 << 16), (0.2, 1), (1.0, 1 << 20)])
def test_pruned_probe_matches_oracle(env, rate, B):
    g, torch, ctx = env
    rng = np.random.default_rng(int(B) + 7)
    host, dtypes = _edge_table(300_000 + 91, rng)
    dev = [torch.from_numpy(c).cuda() for c in host]
    tab = g.Table(dev, 5)
    preds = [[(0, g.RANGE, (400_000, 410_000))],                            # a narrow clustered range
             [(2, g.EQ, (int(host[2][123_456]),))],                         # one value of a sorted int64
             [(0, g.IN, (5, 999_999, 123_457)), (3, g.RANGE, (0.25, 0.5))],
             [(3, g.EQ, (0.0,))], [(1, g.RANGE, (INT32_MIN, INT32_MIN + 1))]]
    zm = g.gace_zonemap_build(ctx, tab)
    try:
        for sub in (preds[:1], preds[:2], preds):
            print("zone probe", rate, B, len(sub), flush=True)
            got = g.gace_probe_selectivity_zm(ctx, tab, zm, sub, 17, rate, B)
            plain = g.gace_probe_selectivity(ctx, tab, sub, 17, rate, B)
            want = oracle.probe_selectivity(host, dtypes, 5, sub, 17, rate, B)
            assert got[0].tolist() == want[0].tolist() == plain[0].tolist()
            assert got[1:3] == want[1:] == plain[1:]
            zmin, zmax = zip(*[oz.zone_minmax(c) for c in host])
            assert got[3] == int(oz.skipped_zones(list(zmin), list(zmax), dtypes, sub).sum())
        assert g.gace_probe_selectivity_zm(ctx, tab, zm, preds[:1], 17, rate, B)[3] > 50
    finally:
        g.gace_zonemap_destroy(zm)


def test_zonemap_belongs_to_its_table(env):
    g, torch, ctx = env
    a = [torch.arange(10_000, dtype=torch.int32, device="cuda")]
    b = [torch.arange(10_000, dtype=torch.int32, device="cuda")]
    zm = g.gace_zonemap_build(ctx, g.Table(a, 1))
    try:
        with pytest.raises(g.GaceError) as e:
            g.gace_probe_selectivity_zm(ctx, g.Table(b, 1), zm, [[(0, g.EQ, (5,))]])
        assert e.value.status == g.GACE_EINVAL
        got = g.gace_probe_selectivity_zm(ctx, g.Table(a, 1), zm, [[(0, g.RANGE, (5000, 5100))]])
        assert got[0].tolist() == [100] and got[3] == 2           # zones 0 and 2 of 3 cannot hold it
    finally:
        g.gace_zonemap_destroy(zm)
    empty = [torch.zeros(0, dtype=torch.int32, device="cuda")]
    zm = g.gace_zonemap_build(ctx, g.Table(empty, 1))
    try:
        got = g.gace_probe_selectivity_zm(ctx, g.Table(empty, 1), zm, [[(0, g.EQ, (5,))]])
        assert got[0].tolist() == [0] and got[1:] == (0, 0, 0)
    finally:
        g.gace_zonemap_destroy(zm)


def test_batched_scans_use_attached_zone_maps(env):
    """Zone maps attached to a context (and to a server) prune shared scans in
    batches: a zone is skipped only when no request of the scan can match in
    it, and every count equals the oracle's with and without the zone map."""
    g, torch, ctx = env
    rng = np.random.default_rng(41)
    host, dtypes = _edge_table(400_000 + 17, rng)
    dev = [torch.from_numpy(c).cuda() for c in host]
    tab = g.Table(dev, 5)
    other = datagen.uniform_i32_table(90_001, 4, 77, 6)
    other_dev = datagen.device_table(other, torch.device("cuda:0"))
    other_host = [c.cpu().numpy() for c in other_dev]
    narrow = [[(0, g.RANGE, (400_000, 410_000))], [(0, g.RANGE, (10, 20)), (3, g.RANGE, (0.1, 0.9))]]
    narrow2 = [[(2, g.EQ, (int(host[2][123_456]),))], [(0, g.IN, (5, 999_999))]]
    wide = [[(1, g.RANGE, (INT32_MIN, INT32_MAX))]]          # can hold in every zone

    def reqs(with_wide):
        out = [(tab, host, dtypes, 5, narrow, 1.0), (tab, host, dtypes, 5, narrow2, 0.5),
               (g.Table(other_dev, 6), other_host, [c.dtype for c in other.cols], 6,
                [[(0, g.RANGE, (100, 300))]], 0.3)]
        if with_wide:
            out.append((tab, host, dtypes, 5, wide, 0.7))
        return out

    def run(spec, c=ctx):
        qs = [g.SelRequest(t, p, 17, rate, 4096) for (t, _, _, _, p, rate) in spec]
        assert g.gace_batch_run(c, qs) == [0] * len(qs)
        return [q.result() for q in qs], g.gace_last_kernel_stats(c)["zones_skipped"]

    def want(spec):
        return [oracle.probe_selectivity(h, d, tid, p, 17, rate, 4096) for (_, h, d, tid, p, rate) in spec]

    zm = g.gace_zonemap_build(ctx, tab)
    try:
        for with_wide in (False, True):
            spec = reqs(with_wide)
            w = want(spec)
            base, z0 = run(spec)
            assert z0 == 0
            g.gace_zonemap_attach(ctx, zm)
            g.gace_zonemap_attach(ctx, zm)                  # a second attach is a no-op
            print("batched zone maps, wide request:", with_wide, flush=True)
            for graph in (True, False):
                g.gace_set_graph(ctx, graph)
                got, zs = run(spec)
                for a, b, c in zip(got, base, w):
                    assert a[0].tolist() == b[0].tolist() == c[0].tolist() and a[1:] == b[1:] == c[1:]
                # the clustered table's narrow predicates skip zones; a request
                # that can match anywhere on the same scan keeps them all
                assert (zs > 0) == (not with_wide), zs
            g.gace_set_graph(ctx, True)
            g.gace_zonemap_detach(ctx, zm)
            assert run(spec)[1] == 0
        with pytest.raises(g.GaceError):
            g.gace_zonemap_detach(ctx, zm)
        # served batches with the zone map attached to the server
        spec = reqs(False)
        w = want(spec)
        srv = g.gace_server_create(0, max_inflight=2, max_batch=8, queue_capacity=64, workspace_bytes=2 << 30)
        try:
            g.gace_server_attach_zonemap(srv, zm)
            qs = [g.SelRequest(t, p, 17, rate, 4096) for (t, _, _, _, p, rate) in spec]
            tickets = [g.gace_server_submit(srv, q) for q in qs]
            assert [g.gace_server_wait(srv, t, 60_000_000_000) for t in tickets] == [0] * len(qs)
            for q, c in zip(qs, w):
                r = q.result()
                assert r[0].tolist() == c[0].tolist() and r[1:] == c[1:]
        finally:
            g.gace_server_destroy(srv)
    finally:
        g.gace_zonemap_destroy(zm)
