"""Zone-map oracle pins (no GPU): the per-zone minima and maxima bound every
value of the zone and are attained; a zone the oracle marks as skippable has
no row satisfying any predicate (checked row by row with the probe oracle);
a zone holding a matching row is never skipped."""
import numpy as np

import oracle
from oracle import zonemap as oz

INT32_MIN, INT32_MAX = -(2**31), 2**31 - 1


def _table(n, rng):
    c0 = np.sort(rng.integers(0, 100_000, n)).astype(np.int32)            # clustered
    c1 = rng.integers(INT32_MIN, INT32_MAX, n, dtype=np.int64).astype(np.int32)
    c2 = (np.sort(rng.integers(-2**40, 2**40, n))).astype(np.int64)
    c3 = rng.random(n).astype(np.float32)
    c3[:5000] = np.nan                                                   # the first zone: NaN only
    c3[9000] = np.float32(-0.0)
    return [c0, c1, c2, c3], [1, 1, 2, 3]


def test_minmax_bounds_and_attained():
    rng = np.random.default_rng(1)
    cols, _ = _table(20_000 + 77, rng)
    for c in cols:
        lo, hi = oz.zone_minmax(c)
        for z in range(lo.size):
            seg = c[z * 4096:(z + 1) * 4096]
            if c.dtype == np.float32:
                seg = seg[~np.isnan(seg)]
            if seg.size == 0:
                assert lo[z] == np.inf and hi[z] == -np.inf
                continue
            assert (seg >= lo[z]).all() and (seg <= hi[z]).all()
            assert lo[z] in seg and hi[z] in seg


def test_skipped_zones_are_sound_and_tight_for_clustered_ranges():
    rng = np.random.default_rng(2)
    cols, dtypes = _table(40_000 + 5, rng)
    zmin, zmax = zip(*[oz.zone_minmax(c) for c in cols])
    preds = [[(0, 1, (30_000, 31_000))], [(2, 2, (int(cols[2][12_345]),))],
             [(0, 3, (5, 99_000)), (3, 1, (0.25, 0.5))], [(3, 2, (0.0,))]]
    skip = oz.skipped_zones(list(zmin), list(zmax), dtypes, preds)
    n = cols[0].shape[0]
    for z in range(skip.size):
        seg = [c[z * 4096:(z + 1) * 4096] for c in cols]
        counts, _, _ = oracle.probe_selectivity(seg, dtypes, 1, preds, 0, 1.0, 4096)
        if skip[z]:
            assert counts.sum() == 0, z          # sound: nothing there can match
    # a clustered range touches few zones: most are skipped
    only = oz.skipped_zones(list(zmin), list(zmax), dtypes, preds[:1])
    assert only.sum() >= skip.size - 2
    # the NaN-only first zone cannot hold the float terms
    assert not oz.term_may(zmin[3][0], zmax[3][0], 2, (0.0,), 3)
    # -0.0 equals +0.0
    z = 9000 // 4096
    assert oz.term_may(zmin[3][z], zmax[3][z], 2, (0.0,), 3)
