"""gace_probe_selectivity_noalloc (the selectivity probe on the library's
static scratch, no context) against gace_probe_selectivity on a context's
workspace and against the oracle: two calls in a row, the second on a
smaller input, so leftovers of the first call in the shared scratch would
show; then a request beyond the scratch's limits fails with GACE_ENOMEM and
leaves its counts untouched."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    torch.cuda.set_device(0)
    import paper_2512_19750_amd as g
    g.lib()
    return g


def _say(*a):
    print(*a, flush=True)


def _case(n_rows, n_preds, rate, B):
    w = datagen.config2(n_rows=n_rows, n_preds=n_preds, rate=rate)
    return w.tables[0], w.sel[0].preds, w.sel[0].spec.seed, rate, B


def test_noalloc_matches_context_path_twice(g):
    import torch
    dev = torch.device("cuda:0")
    ctx = g.gace_create(0, 1 << 30)
    try:
        # a ragged table over many items and 64 predicates, then a much smaller
        # one with fewer predicates and row-level blocks
        for n_rows, n_preds, rate, B in [(3_000_001, 64, 0.3, 4096), (70_001, 9, 0.5, 256)]:
            t, preds, seed, rate, B = _case(n_rows, n_preds, rate, B)
            cols = datagen.device_table(t, dev)
            tab = g.Table(cols, t.table_id)
            _say("noalloc", n_rows, n_preds, rate, B)
            got = g.gace_probe_selectivity_noalloc(tab, preds, seed, rate, B)
            ref = g.gace_probe_selectivity(ctx, tab, preds, seed, rate, B)
            assert got[0].tolist() == ref[0].tolist() and got[1:] == ref[1:]
            host = [c.cpu().numpy() for c in cols]
            want = oracle.probe_selectivity(host, [c.dtype for c in t.cols], t.table_id, preds, seed, rate, B)
            assert got[0].tolist() == want[0].tolist() and got[1:] == want[1:]
    finally:
        g.gace_destroy(ctx)


def test_noalloc_rejects_beyond_scratch(g):
    import torch
    dev = torch.device("cuda:0")
    t = datagen.uniform_i32_table(50_000, 4, 1234, 9)
    cols = datagen.device_table(t, dev)
    rng = np.random.default_rng(5)
    # 8,192 predicates of four RANGE terms compile to a plan of about 4 MB of
    # interval-mask tables alone (128 groups x 4 columns x ~8 KB), more than
    # the scratch's 2 MiB plan region
    preds = [[(c, datagen.RANGE, (lo, lo + int(rng.integers(1, 11))))
              for c, lo in enumerate(int(x) for x in rng.integers(0, 990, 4))] for _ in range(8192)]
    counts = np.full(len(preds), 0xDEADBEEF, dtype=np.uint64)
    with pytest.raises(g.GaceError) as e:
        g.gace_probe_selectivity_noalloc(g.Table(cols, t.table_id), preds, 3, 1.0, 4096, counts=counts)
    assert e.value.status == g.GACE_ENOMEM
    assert "static scratch" in str(e.value)
    assert np.all(counts == 0xDEADBEEF)
    # the scratch still serves a request within its limits afterwards
    small = preds[:64]
    got = g.gace_probe_selectivity_noalloc(g.Table(cols, t.table_id), small, 3, 1.0, 4096)
    host = [c.cpu().numpy() for c in cols]
    want = oracle.probe_selectivity(host, [c.dtype for c in t.cols], t.table_id, small, 3, 1.0, 4096)
    assert got[0].tolist() == want[0].tolist() and got[1:] == want[1:]
