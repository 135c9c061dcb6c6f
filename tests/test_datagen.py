"""The seeded column generator: ranges, laws, determinism, row-offset
consistency.  CPU only (host==device identity is a GPU test)."""
import math

import numpy as np

import datagen


def test_uniform_range_and_mean():
    t = datagen.uniform_i32_table(200_000, 2, 11, 3)
    a, b = datagen.host_table(t)
    assert a.min() >= 0 and a.max() <= 999 and b.min() >= 0 and b.max() <= 999
    assert abs(a.mean() - 499.5) < 6 * 288.7 / math.sqrt(a.size)
    assert not np.array_equal(a, b)


def test_row_offset_and_threads_consistent():
    t = datagen.config2_table(300_000)
    full = datagen.host_table(t, nthreads=1)
    part = datagen.host_table(t, row0=123_457, n=50_000, nthreads=5)
    for f, p in zip(full, part):
        assert np.array_equal(f[123_457:173_457], p)
    again = datagen.host_table(t, nthreads=8)
    for f, g in zip(full, again):
        assert np.array_equal(f, g)


def test_zipf_head_frequencies():
    # bounded Zipf(1.1) on [0, 10^6): P(value r) = (r+1)^-1.1 / H; the ten most
    # frequent values against their expected counts (6 sigma)
    t = datagen.config2_table(1_000_000)
    c0 = datagen.host_column(t.cols[0], t.n_rows)
    assert c0.min() >= 0 and c0.max() < 1_000_000
    r = np.arange(1, 1_000_001, dtype=np.float64)
    p = r ** -1.1
    p /= p.sum()
    cnt = np.bincount(c0[c0 < 10], minlength=10)
    for v in range(10):
        mu = c0.size * p[v]
        assert abs(cnt[v] - mu) <= 6 * math.sqrt(mu * (1 - p[v])), v


def test_correlated_noise_and_other_columns():
    t = datagen.config2_table(200_000)
    c = datagen.host_table(t)
    d = c[1].astype(np.int64) - c[0].astype(np.int64)
    assert d.min() == -50 and d.max() == 50
    hist = np.bincount(d + 50, minlength=101)
    e = d.size / 101
    assert float(((hist - e) ** 2 / e).sum()) < 100 + 6 * math.sqrt(200)
    assert c[2].min() >= 0 and c[2].max() < 10_000
    assert c[4].dtype == np.int64 and c[4].min() >= 0 and c[4].max() < 1_000_000
    assert c[5].min() >= -(1 << 40) and c[5].max() < (1 << 40) and c[5].min() < -(1 << 39)
    for f in (c[6], c[7]):
        assert f.dtype == np.float32 and f.min() >= 0.0 and f.max() < 1.0
        assert np.all((f.astype(np.float64) * 2**24) == np.floor(f.astype(np.float64) * 2**24))


def test_values_at_matches_fill():
    t = datagen.config2_table(10_000)
    rows = np.array([0, 5, 9999, 1234], dtype=np.uint64)
    for c in t.cols:
        col = datagen.host_column(c, t.n_rows)
        v = datagen.host_values_at(c, rows)
        if c.dtype == datagen.F32:
            assert np.array_equal(col.view(np.uint32)[rows.astype(np.int64)].astype(np.int64), v)
        else:
            assert np.array_equal(col[rows.astype(np.int64)].astype(np.int64), v)


def test_workload_recipes_deterministic():
    a, b = datagen.config4(scale=0.001), datagen.config4(scale=0.001)
    assert [t.n_rows for t in a.tables] == [t.n_rows for t in b.tables]
    assert [r.preds for r in a.sel] == [r.preds for r in b.sel]
    assert a.order == b.order
    assert len(a.sel) == 448 and len(a.joins) == 64
    assert all(1 <= len(r.preds) <= 32 for r in a.sel)
    assert all(0.001 <= r.spec.rate <= 1.0 for r in a.sel)
    # one sampling seed per table: requests on a table share it
    seeds = {}
    for r in a.sel:
        seeds.setdefault(r.table, set()).add(r.spec.seed)
    assert all(len(s) == 1 for s in seeds.values())
