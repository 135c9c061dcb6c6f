"""Oracle of the sample-scaled estimates (selectivity, Horvitz-Thompson
cardinality and join size, GEE NDV scale-up) used to turn the probe's exact
sample counts into population estimates.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`.

Definitions:
  * every row of a table is kept with probability p = thr / 2^32
    (thr = floor(rate 2^32); p = 1 at rate 1), since its block is;
  * ratio estimator of the selectivity: count / sampled rows (S_probe, Eq. 2);
  * Horvitz-Thompson: each sampled row stands for 1 / p rows, each sampled
    pair of an R row and an S row (independent samples) for 1 / (p_R p_S)
    pairs;
  * GEE (Charikar, Chaudhuri, Motwani, Narasayya, PODS 2000): the distinct
    values seen once in a sample of r of n rows are scaled by sqrt(n / r),
    those seen more often are counted once.
All in binary64, in the order written.
"""
from __future__ import annotations

import math

from . import threshold


def inclusion(rate: float) -> float:
    thr = threshold(rate)
    return 1.0 if thr >= 1 << 32 else thr / 4294967296.0


def gee(n: int, r: int, d: int, f1: int) -> float:
    if r == 0:
        return 0.0
    return math.sqrt(n / r) * f1 + (d - f1)


def sel_estimate(count: int, sampled: int, n_rows: int, rate: float) -> dict:
    p = inclusion(rate)
    sel = count / sampled if sampled else math.nan
    return dict(p=p, sel=sel, card=sel * n_rows if sampled else math.nan,
                card_ht=count / p if p > 0 else math.nan)


def join_estimate(res: dict, n_R: int, rate_R: float, n_S: int, rate_S: float) -> dict:
    pr, ps = inclusion(rate_R), inclusion(rate_S)
    return dict(p_R=pr, p_S=ps, join_ht=res["join_card"] / (pr * ps) if pr > 0 and ps > 0 else math.nan,
                ndv_R=gee(n_R, res["n_R"], res["ndv_R"], res["f1_R"]),
                ndv_S=gee(n_S, res["n_S"], res["ndv_S"], res["f1_S"]))
