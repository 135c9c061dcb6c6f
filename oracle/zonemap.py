"""Oracle of zone maps (block-level summaries, Sec. III-B): per column and
zone of 4096 rows the smallest and largest value, and the zones on which no
candidate condition can hold.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`.

Definitions (readings):
  * float32 zones summarise their non-NaN values (NaN satisfies no term); a
    zone of NaNs only is empty: min = +inf, max = -inf;
  * a term can hold on a zone iff some value v with min <= v <= max satisfies
    it: RANGE [lo, hi) iff max >= lo and min < hi (and the zone is not
    empty); EQ / IN iff one of the values lies in [min, max];
  * a predicate can hold iff each of its terms can; a zone is skipped iff no
    predicate can hold.  Integers compare in int64, floats as binary32.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

ZONE_ROWS = 4096
F32, RANGE = 3, 1


def zone_minmax(col: np.ndarray):
    n = col.shape[0]
    nz = (n + ZONE_ROWS - 1) // ZONE_ROWS
    lo = np.empty(nz, dtype=col.dtype)
    hi = np.empty(nz, dtype=col.dtype)
    for z in range(nz):
        seg = col[z * ZONE_ROWS:(z + 1) * ZONE_ROWS]
        if col.dtype == np.float32:
            seg = seg[~np.isnan(seg)]
            if seg.size == 0:
                lo[z], hi[z] = np.float32(np.inf), np.float32(-np.inf)
                continue
        lo[z], hi[z] = seg.min(), seg.max()
    return lo, hi


def term_may(lo, hi, op: int, vals: Sequence[int], dtype: int) -> bool:
    if dtype == F32:
        lo, hi = np.float32(lo), np.float32(hi)
        vs = [np.float32(v) for v in vals]
        if op == RANGE:
            return bool(hi >= vs[0] and lo < vs[1] and lo <= hi)
        return any(lo <= v <= hi for v in vs)
    lo, hi = int(lo), int(hi)
    if op == RANGE:
        return hi >= vals[0] and lo < vals[1]
    return any(lo <= v <= hi for v in vals)


def skipped_zones(zmin: List[np.ndarray], zmax: List[np.ndarray], dtypes: Sequence[int], preds) -> np.ndarray:
    """Boolean per zone: True when no predicate can hold on it.  preds as the
    probe's lists of (col, op, values) terms (float32 columns: float values)."""
    nz = zmin[0].shape[0] if zmin else 0
    out = np.zeros(nz, dtype=bool)
    for z in range(nz):
        may = False
        for p in preds:
            if all(term_may(zmin[c][z], zmax[c][z], op, vals, dtypes[c]) for c, op, vals in p):
                may = True
                break
        out[z] = not may
    return out
