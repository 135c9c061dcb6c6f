"""Failure paths of the C ABI on the GPU, each forced from the host so every
kernel still exits normally: a join phase wait that gives up (spin limit 0)
fails that join with GACE_EDEVICE while the rest of the batch completes; a
workspace too small for a join's partitions, or a plan too large for its
region, fails with GACE_ENOMEM; a failed request's outputs are untouched.
The results that do come back equal the oracle's."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

SENTINEL = 0xDEADBEEF


@pytest.fixture(scope="module")
def g():
    import torch
    torch.cuda.set_device(0)
    import paper_2512_19750_amd as g
    g.lib()
    return g


def _say(*a):
    print(*a, flush=True)


def _join_workload(n_r, n_s, dom, rate, seed):
    r, s = datagen.join_pair(n_r, n_s, dom, seed, 31, 32)
    return r, s, datagen.SampleSpec(seed + 1, rate, 4096), datagen.SampleSpec(seed + 2, rate, 4096)


def _mark(q):
    """Fill a request's outputs with a sentinel, so an untouched output shows."""
    if hasattr(q, "out"):
        for f, _ in q.out._fields_:
            setattr(q.out, f, SENTINEL)
    else:
        q.counts[:] = SENTINEL


def _untouched(q):
    if hasattr(q, "out"):
        return all(getattr(q.out, f) == SENTINEL for f, _ in q.out._fields_)
    return bool(np.all(q.counts == SENTINEL))


def test_wait_give_up_fails_only_the_join(g):
    import torch
    dev = torch.device("cuda:0")
    r, s, sr, ss = _join_workload(600_000, 200_000, 100_000, 1.0, 71)
    kr = datagen.device_column(r.cols[0], r.n_rows, dev)
    ks = datagen.device_column(s.cols[0], s.n_rows, dev)
    w = datagen.config1(200_000)
    t = w.tables[0]
    cols = datagen.device_table(t, dev)
    host = [c.cpu().numpy() for c in cols]
    preds = w.sel[0].preds
    ctx = g.gace_create(0, 2 << 30)
    try:
        want_join = oracle.join_freq(kr.cpu().numpy(), r.table_id, sr.seed, sr.rate, 4096,
                                     ks.cpu().numpy(), s.table_id, ss.seed, ss.rate, 4096)
        want_sel = oracle.probe_selectivity(host, [c.dtype for c in t.cols], t.table_id, preds, 5, 1.0, 4096)
        for graph in (False, True):
            g.gace_set_graph(ctx, graph)
            g.gace_set_spin_limit(ctx, 0)      # every join phase wait gives up at once
            sel = g.SelRequest(g.Table(cols, t.table_id), preds, 5, 1.0, 4096)
            jn = g.JoinRequest(g.Keys(kr, r.table_id, sr.seed, sr.rate, 4096),
                               g.Keys(ks, s.table_id, ss.seed, ss.rate, 4096))
            _mark(sel)
            _mark(jn)
            _say("spin limit 0, graph", graph)
            st = g.gace_batch_run(ctx, [sel, jn], raise_on_error=False)
            assert st == [g.GACE_OK, g.GACE_EDEVICE], st
            assert _untouched(jn)
            assert sel.result()[0].tolist() == want_sel[0].tolist() and sel.result()[1:] == want_sel[1:]
            # the default bound: the same join completes and equals the oracle
            g.gace_set_spin_limit(ctx, 1 << 24)
            _say("default spin limit, graph", graph)
            assert g.gace_batch_run(ctx, [jn]) == [g.GACE_OK]
            assert jn.result() == want_join
    finally:
        g.gace_destroy(ctx)


def test_small_workspace_join_enomem_outputs_untouched(g):
    import torch
    dev = torch.device("cuda:0")
    # 8e6 keys at rate 1: two partitioning buffers of 64 MB each, more than
    # the arena of the smallest workspace (64 MiB beyond the fixed regions)
    r, s, sr, ss = _join_workload(6_000_000, 2_000_000, 1_000_000, 1.0, 91)
    kr = datagen.device_column(r.cols[0], r.n_rows, dev)
    ks = datagen.device_column(s.cols[0], s.n_rows, dev)
    # the smallest workspace gace_create accepts: its fixed regions plus a
    # 64 MiB arena (found by trying sizes upwards)
    ctx = None
    for mib in range(100, 200, 4):
        try:
            ctx = g.gace_create(0, mib << 20)
            break
        except g.GaceError:
            continue
    assert ctx is not None
    try:
        R = g.Keys(kr, r.table_id, sr.seed, sr.rate, 4096)
        S = g.Keys(ks, s.table_id, ss.seed, ss.rate, 4096)
        with pytest.raises(g.GaceError) as e:
            g.gace_join_freq(ctx, R, S)
        assert e.value.status == g.GACE_ENOMEM, e.value
        assert "arena" in str(e.value) or "workspace" in str(e.value)
        w = datagen.config1(100_000)
        t = w.tables[0]
        cols = datagen.device_table(t, dev)
        sel = g.SelRequest(g.Table(cols, t.table_id), w.sel[0].preds, 1, 1.0, 4096)
        jn = g.JoinRequest(R, S)
        _mark(sel)
        _mark(jn)
        st = g.gace_batch_run(ctx, [jn, sel], raise_on_error=False)
        assert st == [g.GACE_ENOMEM, g.GACE_OK], st
        assert _untouched(jn)
        host = [c.cpu().numpy() for c in cols]
        want = oracle.probe_selectivity(host, [c.dtype for c in t.cols], t.table_id, w.sel[0].preds, 1, 1.0, 4096)
        assert sel.result()[0].tolist() == want[0].tolist()
    finally:
        g.gace_destroy(ctx)


def test_plan_too_large_enomem_outputs_untouched(g):
    import torch
    dev = torch.device("cuda:0")
    t = datagen.uniform_i32_table(50_000, 4, 1234, 9)
    cols = datagen.device_table(t, dev)
    rng = np.random.default_rng(5)
    # 65,536 predicates of four wide RANGE terms: about 1,024 groups x 4
    # columns of 8 KB interval-mask tables, more than the 16 MiB plan region
    preds = []
    for _ in range(65536):
        p = []
        for c in range(4):
            lo = int(rng.integers(0, 990))
            p.append((c, datagen.RANGE, (lo, lo + int(rng.integers(1, 11)))))
        preds.append(p)
    ctx = g.gace_create(0, 1 << 30)
    try:
        sel = g.SelRequest(g.Table(cols, t.table_id), preds, 3, 1.0, 4096)
        _mark(sel)
        st = g.gace_batch_run(ctx, [sel], raise_on_error=False)
        assert st == [g.GACE_ENOMEM], st
        assert "plan" in g.last_error()
        assert _untouched(sel)
        with pytest.raises(g.GaceError) as e:
            g.gace_probe_selectivity(ctx, g.Table(cols, t.table_id), preds, 3, 1.0, 4096)
        assert e.value.status == g.GACE_ENOMEM
    finally:
        g.gace_destroy(ctx)
