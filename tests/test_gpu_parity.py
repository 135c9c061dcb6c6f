"""GPU parity: every count, NDV and join size from the HIP path (called through
the C ABI) equals the CPU oracle's, bit for bit in uint64."""
import math
import os

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

INT32_MIN, INT32_MAX = -(2**31), 2**31 - 1
INT64_MIN, INT64_MAX = -(2**63), 2**63 - 1


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def g():
    import paper_2512_19750_amd as g
    g.lib()
    return g


@pytest.fixture(scope="module")
def ctx(g, torch_dev):
    c = g.gace_create(0, 8 << 30)
    yield c
    g.gace_destroy(c)


def _say(*a):
    print(*a, flush=True)


def _tensors(host_cols, dev):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(c)).to(dev) for c in host_cols]


# ---------------------------------------------------------------- generator
def test_device_generator_matches_host(torch_dev):
    t = datagen.config2_table(300_000)
    for c in t.cols:
        d = datagen.device_column(c, 5000, torch_dev, row0=123_456).cpu().numpy()
        h = datagen.host_column(c, 5000, row0=123_456)
        assert d.tobytes() == h.tobytes()
    r, s = datagen.join_pair(1000, 1000, 10_000_000, 99, 3, 4)
    for tb in (r, s):
        d = datagen.device_column(tb.cols[0], 100_000, torch_dev, row0=7).cpu().numpy()
        assert d.tobytes() == datagen.host_column(tb.cols[0], 100_000, row0=7).tobytes()


# ---------------------------------------------------------------- selectivity
def _edge_table(rng, n):
    c0 = rng.integers(-5, 6, size=n).astype(np.int32)
    c0[rng.random(n) < 0.05] = INT32_MIN
    c0[rng.random(n) < 0.05] = INT32_MAX
    c1 = rng.integers(-3, 4, size=n).astype(np.int64)
    c1[rng.random(n) < 0.05] = INT64_MIN
    c1[rng.random(n) < 0.05] = INT64_MAX
    c2 = rng.choice(np.array([-1.5, -0.0, 0.0, 0.25, 0.5, 1.0, np.nan, -np.nan, np.inf, -np.inf], dtype=np.float32),
                    size=n)
    c3 = rng.integers(0, 1000, size=n).astype(np.int32)
    return [c0, c1, c2, c3], [1, 2, 3, 1]


def _edge_preds(rng, n_preds):
    pools = {0: [INT32_MIN, -5, -1, 0, 1, 5, INT32_MAX, -(2**40), 2**40],
             1: [INT64_MIN, -3, 0, 3, INT64_MAX],
             2: [-1.5, -0.0, 0.0, 0.25, 1.0, float("inf"), float("-inf")], 3: [0, 10, 500, 999, 1000]}
    preds = []
    for _ in range(n_preds):
        terms = []
        for _ in range(int(rng.integers(1, 6))):
            c = int(rng.integers(0, 4))
            op = int(rng.integers(1, 4))
            pool = pools[c]
            if op == 1:
                a, b = rng.choice(len(pool), 2)
                terms.append((c, op, (pool[a], pool[b])))
            elif op == 2:
                terms.append((c, op, (pool[int(rng.integers(len(pool)))],)))
            else:
                terms.append((c, op, tuple(pool[int(i)] for i in rng.integers(0, len(pool), int(rng.integers(1, 9))))))
        preds.append(terms)
    return preds


@pytest.mark.parametrize("seed", range(8))
def test_edge_values_vs_oracle(g, ctx, torch_dev, seed):
    rng = np.random.default_rng(1000 + seed)
    n = [1, 63, 4096, 3 * 4096 + 17, 50_001, 100_000, 7, 70_000][seed]
    cols, dtypes = _edge_table(rng, n)
    n_preds = [1, 5, 64, 65, 130, 200, 3, 64][seed]
    preds = _edge_preds(rng, n_preds)
    B = [1, 4, 4096, 64, 1 << 20, 256, 2, 128][seed]
    rate = [1.0, 0.5, 0.13, 1.0, 1.0, 0.7, 0.0, 0.02][seed]
    _say("edge case", seed, "n", n, "preds", n_preds, "B", B, "rate", rate)
    table = g.Table(_tensors(cols, torch_dev), 40 + seed)
    got = g.gace_probe_selectivity(ctx, table, preds, seed=77 + seed, rate=rate, block_rows=B)
    want = oracle.probe_selectivity(cols, dtypes, 40 + seed, preds, 77 + seed, rate, B)
    assert got[1:] == want[1:]
    assert got[0].tolist() == want[0].tolist()


@pytest.mark.parametrize("B,rate", [(1, 0.3), (1, 0.0002), (2, 0.05), (8, 0.0015), (8, 0.003), (512, 0.2),
                                    (2048, 0.45), (2048, 0.55)])
def test_small_blocks_vs_oracle(g, ctx, torch_dev, B, rate):
    """Blocks under 4096 rows on both sides of the switch between the
    block-by-block scan and the row-by-row tile scan (one kept block per
    4096 rows expected: rate = B / 4096), over two predicate groups, a
    ragged last tile and a partial last block."""
    rng = np.random.default_rng(B * 1000 + int(rate * 1e4))
    n = 5 * 4096 * 3 + 1237
    cols, dtypes = _edge_table(rng, n)
    preds = _edge_preds(rng, 70)
    _say("small blocks", B, rate)
    table = g.Table(_tensors(cols, torch_dev), 61)
    got = g.gace_probe_selectivity(ctx, table, preds, seed=5, rate=rate, block_rows=B)
    want = oracle.probe_selectivity(cols, dtypes, 61, preds, 5, rate, B)
    assert got[1:] == want[1:]
    assert got[0].tolist() == want[0].tolist()


@pytest.mark.parametrize("mode", [1, 2])
def test_count_modes_agree(g, torch_dev, mode):
    rng = np.random.default_rng(5)
    cols, dtypes = _edge_table(rng, 40_000)
    preds = _edge_preds(rng, 100)
    table = g.Table(_tensors(cols, torch_dev), 9)
    c = g.gace_create(0, 1 << 30)
    try:
        g.gace_set_schedule(c, count_mode=mode)
        got = g.gace_probe_selectivity(c, table, preds, seed=3, rate=0.5, block_rows=64)
    finally:
        g.gace_destroy(c)
    want = oracle.probe_selectivity(cols, dtypes, 9, preds, 3, 0.5, 64)
    assert got[0].tolist() == want[0].tolist() and got[1:] == want[1:]


def test_config1_full(g, ctx, torch_dev):
    w = datagen.config1()
    t = w.tables[0]
    cols = datagen.device_table(t, torch_dev)
    req = w.sel[0]
    got = g.gace_probe_selectivity(ctx, g.Table(cols, t.table_id), req.preds, req.spec.seed, 1.0, 4096)
    want = oracle.sel_request(w, 0)
    assert got[0].tolist() == want[0].tolist() and got[1] == want[1] == 1_000_000
    assert abs(int(got[0][0]) - 100_000) <= 1800


@pytest.mark.parametrize("n_rows,rate,B", [(2_000_000, 1.0, 4096), (2_000_000, 0.01, 4096), (1_000_003, 0.2, 512)])
def test_config2_reduced(g, ctx, torch_dev, n_rows, rate, B):
    w = datagen.config2(n_rows=n_rows, rate=rate)
    t = w.tables[0]
    req = w.sel[0]
    _say("config2 reduced", n_rows, rate, B)
    cols = datagen.device_table(t, torch_dev)
    got = g.gace_probe_selectivity(ctx, g.Table(cols, t.table_id), req.preds, req.spec.seed, rate, B)
    host = [c.cpu().numpy() for c in cols]
    want = oracle.probe_selectivity(host, [c.dtype for c in t.cols], t.table_id, req.preds, req.spec.seed, rate, B)
    assert got[0].tolist() == want[0].tolist() and got[1:] == want[1:]


def test_config2_full(g, ctx, torch_dev):
    # 10^8 rows x 8 columns, 64 predicates, 1 % block sampling: the oracle
    # regenerates only the kept blocks
    w = datagen.config2()
    t = w.tables[0]
    req = w.sel[0]
    cols = datagen.device_table(t, torch_dev)
    got = g.gace_probe_selectivity(ctx, g.Table(cols, t.table_id), req.preds, req.spec.seed, req.spec.rate, 4096)
    del cols
    want = oracle.sel_request(w, 0)
    assert got[1:] == want[1:]
    assert got[0].tolist() == want[0].tolist()
    # invariants that hold at any size: the sample is ~1 % of 24,415 blocks
    assert abs(got[2] - 244.15) < 6 * math.sqrt(244.15)


# ---------------------------------------------------------------- joins
def _join(g, ctx, kr, ks, tr, ts, sr, ss, rr, rs, br=4096, bs=4096):
    return g.gace_join_freq(ctx, g.Keys(kr, tr, sr, rr, br), g.Keys(ks, ts, ss, rs, bs))


@pytest.mark.parametrize("case", range(6))
def test_join_small_vs_oracle(g, ctx, torch_dev, case):
    import torch
    rng = np.random.default_rng(200 + case)
    nr = [0, 1, 1000, 5000, 100_000, 300_000][case]
    ns = [10, 0, 2000, 5000, 50_000, 100_000][case]
    dom = [5, 5, 50, 1 << 62, 1000, 40_000][case]
    r = rng.integers(-dom, dom, size=nr, dtype=np.int64)
    s = rng.integers(-dom, dom, size=ns, dtype=np.int64)
    if nr:
        r[rng.random(nr) < 0.02] = INT64_MIN     # the table's sentinel value is a real key too
        r[rng.random(nr) < 0.02] = INT64_MAX
    if ns:
        s[rng.random(ns) < 0.02] = INT64_MIN
        s[rng.random(ns) < 0.01] = -1
    B = [1, 2, 64, 4096, 512, 4096][case]
    rate = [1.0, 1.0, 0.5, 1.0, 0.3, 0.05][case]
    _say("join case", case, nr, ns, B, rate)
    kr = torch.from_numpy(r).to(torch_dev)
    ks = torch.from_numpy(s).to(torch_dev)
    got = _join(g, ctx, kr, ks, 5, 6, 17, 19, rate, rate, B, B)
    want = oracle.join_freq(r, 5, 17, rate, B, s, 6, 19, rate, B)
    assert got == want


@pytest.mark.parametrize("shift,nr,ns,B,rate", [(0, 100_001, 30_001, 2, 0.5), (0, 100_001, 30_001, 4096, 1.0),
                                                 (1, 100_001, 30_001, 4096, 1.0), (1, 100_000, 30_000, 64, 0.7),
                                                 (0, 1, 3, 2, 1.0)])
def test_join_key_alignment_and_odd_lengths(g, ctx, torch_dev, shift, nr, ns, B, rate):
    """Key columns that are only 8-byte aligned (a view one element into a
    tensor, which the ABI allows) and odd lengths, whose last row ends the
    last block."""
    import torch
    rng = np.random.default_rng(nr + 7 * B + shift)
    r = rng.integers(-3000, 3000, size=nr + shift, dtype=np.int64)
    s = rng.integers(-3000, 3000, size=ns + shift, dtype=np.int64)
    r[-1], s[-1] = 2999, 2999          # the last rows pair with each other
    _say("join alignment", shift, nr, ns, B, rate)
    kr_full = torch.from_numpy(r).to(torch_dev)
    ks_full = torch.from_numpy(s).to(torch_dev)
    kr, ks = kr_full[shift:], ks_full[shift:]
    assert (kr.data_ptr() % 16 == 0) == (shift == 0)
    got = _join(g, ctx, kr, ks, 5, 6, 41, 43, rate, rate, B, B)
    assert got == oracle.join_freq(r[shift:], 5, 41, rate, B, s[shift:], 6, 43, rate, B)


@pytest.mark.parametrize("cache", [256, 4096])
def test_join_cache_settings_agree(g, torch_dev, cache):
    import torch
    w = datagen.config3(rate=1.0, n_r=2_000_000, n_s=500_000, domain=100_000)
    jr = w.joins[0]
    kr = datagen.device_column(jr.r.cols[0], jr.r.n_rows, torch_dev)
    ks = datagen.device_column(jr.s.cols[0], jr.s.n_rows, torch_dev)
    c = g.gace_create(0, 2 << 30)
    try:
        g.gace_set_schedule(c, join_part_keys=cache)
        got = _join(g, c, kr, ks, jr.r.table_id, jr.s.table_id, jr.spec_r.seed, jr.spec_s.seed, 1.0, 1.0)
    finally:
        g.gace_destroy(c)
    assert got == oracle.join_request(w, 0)


@pytest.mark.parametrize("B,rate,part", [(1, 0.5, 1024), (16, 0.7, 256), (512, 1.0, 128), (4096, 1.0, 256),
                                          (1 << 16, 0.6, 1024)])
def test_join_two_pass_vs_oracle(g, torch_dev, B, rate, part):
    """Wide fan-outs (two partitioning passes) over kept-block streams of
    several block sizes, skewed keys and the sentinel value."""
    import torch
    rng = np.random.default_rng(B * 7 + part)
    nr, ns = 1_500_000, 600_000
    r = (rng.zipf(1.2, nr) % 300_000).astype(np.int64) * 7919 - 123_456
    s = rng.integers(-50_000, 400_000, size=ns, dtype=np.int64) * 7919 - 123_456
    r[rng.random(nr) < 0.001] = INT64_MIN
    s[rng.random(ns) < 0.001] = INT64_MIN
    _say("two-pass join", B, rate, part)
    kr = torch.from_numpy(r).to(torch_dev)
    ks = torch.from_numpy(s).to(torch_dev)
    c = g.gace_create(0, 2 << 30)
    try:
        g.gace_set_schedule(c, join_part_keys=part)
        got = _join(g, c, kr, ks, 8, 9, 23, 29, rate, rate, B, B)
    finally:
        g.gace_destroy(c)
    assert got == oracle.join_freq(r, 8, 23, rate, B, s, 9, 29, rate, B)


@pytest.mark.parametrize("rate", [1.0, 0.05])
def test_config3_reduced(g, ctx, torch_dev, rate):
    w = datagen.config3(rate=rate, n_r=20_000_000, n_s=5_000_000, domain=1_000_000)
    jr = w.joins[0]
    _say("config3 reduced rate", rate)
    kr = datagen.device_column(jr.r.cols[0], jr.r.n_rows, torch_dev)
    ks = datagen.device_column(jr.s.cols[0], jr.s.n_rows, torch_dev)
    got = _join(g, ctx, kr, ks, jr.r.table_id, jr.s.table_id, jr.spec_r.seed, jr.spec_s.seed, rate, rate)
    assert got == oracle.join_request(w, 0)


def test_config3_full_rate5(g, ctx, torch_dev):
    w = datagen.config3(rate=0.05)
    jr = w.joins[0]
    kr = datagen.device_column(jr.r.cols[0], jr.r.n_rows, torch_dev)
    ks = datagen.device_column(jr.s.cols[0], jr.s.n_rows, torch_dev)
    got = _join(g, ctx, kr, ks, jr.r.table_id, jr.s.table_id, jr.spec_r.seed, jr.spec_s.seed, 0.05, 0.05)
    del kr, ks
    assert got == oracle.join_request(w, 0, nthreads=16)


def test_config3_full_rate1(g, ctx, torch_dev):
    w = datagen.config3(rate=1.0)
    jr = w.joins[0]
    kr = datagen.device_column(jr.r.cols[0], jr.r.n_rows, torch_dev)
    ks = datagen.device_column(jr.s.cols[0], jr.s.n_rows, torch_dev)
    got = _join(g, ctx, kr, ks, jr.r.table_id, jr.s.table_id, jr.spec_r.seed, jr.spec_s.seed, 1.0, 1.0)
    del kr, ks
    # closed forms of the iid law (see the oracle pins): E join = n_R n_S / N
    assert got["n_R"] == 200_000_000 and got["n_S"] == 50_000_000
    assert abs(got["ndv_S"] - 9_932_621) < 6 * 259
    assert abs(got["join_card"] - 1e9) < 0.25e9
    assert got == oracle.join_request(w, 0, nthreads=16)


# ---------------------------------------------------------------- batch
def _materialise(w, dev):
    tabs = []
    for t in w.tables:
        tabs.append(datagen.device_table(t, dev))
    keys = []
    for j in w.joins:
        keys.append((datagen.device_column(j.r.cols[0], j.r.n_rows, dev),
                     datagen.device_column(j.s.cols[0], j.s.n_rows, dev)))
    return tabs, keys


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


def test_batch_matches_oracle_and_plain(g, ctx, torch_dev):
    w = datagen.config4(scale=0.004, n_sel=96, n_join=12)
    tabs, keys = _materialise(w, torch_dev)
    reqs = _requests(g, w, tabs, keys)
    st = g.gace_batch_run(ctx, reqs)
    assert all(s == 0 for s in st)
    for (kind, i), q in zip(w.order, reqs):
        if kind == "sel":
            want = oracle.sel_request(w, i)
            got = q.result()
            assert got[0].tolist() == want[0].tolist() and got[1:] == want[1:], ("sel", i)
            alone = g.gace_probe_selectivity(ctx, q.table, q.preds, q.seed, q.rate, q.block_rows)
            assert alone[0].tolist() == got[0].tolist() and alone[1:] == got[1:]
        else:
            want = oracle.join_request(w, i)
            assert q.result() == want, ("join", i)
            assert g.gace_join_freq(ctx, q.R, q.S) == want


def test_config4_full_batch_vs_oracle(g, torch_dev):
    """The benchmark's workload at full size (16 tables, 448 selectivity and
    64 join requests, 50 GB resident), run as one batch: every one of the 512
    results equals the oracle's, bit for bit, in both launch modes (graph
    replay, twice, and direct launch with per-kernel events), and each
    request run alone on the plain path gives the same result.  The oracle's
    results come from tests/golden/c4_expected.txt, written by
    tests/golden/make_expected.py from oracle/ and the datagen recipes
    alone; its fingerprint ties it to this workload definition."""
    import sys
    import torch
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_expected
    w = datagen.config4()
    want = make_expected.load("c4", w)
    assert len(want) == len(set(w.order)) == 512
    tabs, keys = _materialise(w, torch_dev)
    torch.cuda.synchronize()
    reqs = _requests(g, w, tabs, keys)
    free_b, _ = torch.cuda.mem_get_info()
    c = g.gace_create(0, int(min(free_b * 0.6, 48 << 30)))     # the benchmark's workspace

    def check(tag):
        bad = []
        for key, q in zip(w.order, reqs):
            r = q.result()
            exp = want[key]
            if key[0] == "join":
                if r != exp:
                    bad.append((key, r, exp))
            elif (r[0].tolist(), r[1], r[2]) != exp:
                bad.append((key, (r[0].tolist(), r[1], r[2]), exp))
        assert not bad, (tag, len(bad), bad[:3])

    try:
        for graph, reps in ((True, 2), (False, 1)):
            g.gace_set_graph(c, graph)
            for rep in range(reps):
                _say("config4 full batch, graph replay" if graph else "config4 full batch, direct launch", rep)
                assert all(s == 0 for s in g.gace_batch_run(c, reqs))
                check(("graph" if graph else "direct", rep))
        assert g.gace_last_kernel_stats(c)["timed"]
        for key, q in zip(w.order, reqs):
            if key[0] == "join":
                assert g.gace_join_freq(c, q.R, q.S) == want[key], key
            else:
                cnt, n, k = g.gace_probe_selectivity(c, q.table, q.preds, q.seed, q.rate, q.block_rows)
                assert (cnt.tolist(), n, k) == want[key], key
    finally:
        g.gace_destroy(c)


def test_batch_repeatable_and_schedules_agree(g, torch_dev):
    w = datagen.config4(scale=0.002, n_sel=64, n_join=6, seed_offset=3)
    tabs, keys = _materialise(w, torch_dev)
    c = g.gace_create(0, 2 << 30)
    try:
        results = []
        for sched in [dict(), dict(wgs_per_cu=1, item_rows=16384), dict(wgs_per_cu=3, count_mode=1, item_rows=262144),
                      dict(count_mode=2, join_part_keys=512)]:
            if sched:
                g.gace_set_schedule(c, **sched)
            for rep in range(2):
                reqs = _requests(g, w, tabs, keys)
                g.gace_batch_run(c, reqs)
                results.append([q.result() if isinstance(q, g.JoinRequest) else
                                (q.result()[0].tolist(), q.result()[1:]) for q in reqs])
        # direct launches with per-kernel timing events give the same results
        g.gace_set_graph(c, False)
        reqs = _requests(g, w, tabs, keys)
        g.gace_batch_run(c, reqs)
        results.append([q.result() if isinstance(q, g.JoinRequest) else
                        (q.result()[0].tolist(), q.result()[1:]) for q in reqs])
        ks = g.gace_last_kernel_stats(c)
        assert ks["timed"] and ks["scan_ms"] > 0 and ks["join_ms"] > 0
        assert ks["scan_alg_bytes"] > 0 and ks["join_alg_bytes"] > 0
        # a graph replay carries the same timing events as external event nodes
        g.gace_set_graph(c, True)
        g.gace_batch_run(c, _requests(g, w, tabs, keys))
        ks = g.gace_last_kernel_stats(c)
        assert ks["timed"] and ks["scan_ms"] > 0 and ks["join_ms"] > 0
        for r in results[1:]:
            assert r == results[0]
    finally:
        g.gace_destroy(c)


def test_batch_kinds_in_both_launch_modes(g, torch_dev):
    """Batches of only selectivity requests, only joins, and both, each
    replayed from its own captured graph and launched directly: every result
    equals the plain path's, replay after replay."""
    w = datagen.config4(scale=0.002, n_sel=30, n_join=4, seed_offset=41)
    tabs, keys = _materialise(w, torch_dev)
    c = g.gace_create(0, 2 << 30)
    try:
        def res(q):
            return q.result() if isinstance(q, g.JoinRequest) else (q.result()[0].tolist(), q.result()[1:])
        base = {}
        for kind, i in w.order:
            q = _requests(g, w, tabs, keys)[w.order.index((kind, i))]
            if kind == "sel":
                cnt, n, k = g.gace_probe_selectivity(c, q.table, q.preds, q.seed, q.rate, q.block_rows)
                base[(kind, i)] = (cnt.tolist(), (n, k))
            else:
                base[(kind, i)] = g.gace_join_freq(c, q.R, q.S)
        for graph in (True, False, True):
            g.gace_set_graph(c, graph)
            for pick in ("sel", "join", None):
                order = [o for o in w.order if pick is None or o[0] == pick]
                all_reqs = _requests(g, w, tabs, keys)
                reqs = [all_reqs[w.order.index(o)] for o in order]
                for rep in range(2):
                    g.gace_batch_run(c, reqs)
                    for o, q in zip(order, reqs):
                        assert res(q) == base[o], (graph, pick, rep, o)
    finally:
        g.gace_destroy(c)


def test_batch_invalid_request_fails_alone(g, ctx, torch_dev):
    import torch
    cols = [torch.arange(10_000, dtype=torch.int32, device=torch_dev)]
    t = g.Table(cols, 1)
    good = g.SelRequest(t, [[(0, g.RANGE, (10, 20))]])
    bad = g.SelRequest(t, [[(3, g.RANGE, (10, 20))]])
    bad.counts[:] = 12345
    st = g.gace_batch_run(ctx, [good, bad], raise_on_error=False)
    assert st == [0, g.GACE_EINVAL]
    assert good.result()[0].tolist() == [10]
    assert bad.counts[0] == 12345          # outputs untouched on failure
