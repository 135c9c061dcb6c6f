"""Sample-scaled estimates (no GPU).  The oracle (oracle/estimators.py) is
pinned to what makes each estimator right: Horvitz-Thompson is unbiased under
the block-Bernoulli design (checked by enumerating every keep pattern of tiny
tables with its exact probability), GEE reduces to its closed forms and stays
within its ratio-error guarantee; the library then equals the oracle bit for
bit on random counts."""
import itertools
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_2512_19750_amd as g
from oracle import estimators as oe


def _p_exact(rate):
    thr = oracle.threshold(rate)
    return Fraction(1) if thr >= 1 << 32 else Fraction(thr, 1 << 32)


@pytest.mark.parametrize("rate", [0.3, 0.5, 0.77])
def test_ht_cardinality_is_unbiased_over_all_keep_patterns(rate):
    per_block = [3, 0, 7, 1, 4]          # matching rows in each of 5 blocks
    p = _p_exact(rate)
    expect = Fraction(0)
    for keep in itertools.product([0, 1], repeat=len(per_block)):
        prob = Fraction(1)
        for k in keep:
            prob *= p if k else 1 - p
        count = sum(c for c, k in zip(per_block, keep) if k)
        expect += prob * Fraction(oe.sel_estimate(count, 1, 10, rate)["card_ht"])
    assert float(expect) == pytest.approx(sum(per_block), rel=1e-12)


def test_ht_join_is_unbiased_over_all_keep_patterns():
    R = [[1, 1, 2], [3], [2, 2]]          # keys per block
    S = [[1], [2, 3, 3], [4, 1]]
    rr, rs = 0.4, 0.65
    pr, ps = _p_exact(rr), _p_exact(rs)
    truth = sum(a == b for blk in R for a in blk for sb in S for b in sb)
    expect = Fraction(0)
    for kr in itertools.product([0, 1], repeat=3):
        for ks in itertools.product([0, 1], repeat=3):
            prob = Fraction(1)
            for k in kr:
                prob *= pr if k else 1 - pr
            for k in ks:
                prob *= ps if k else 1 - ps
            rk = [x for blk, k in zip(R, kr) if k for x in blk]
            sk = [x for blk, k in zip(S, ks) if k for x in blk]
            join = sum(a == b for a in rk for b in sk)
            res = dict(join_card=join, n_R=len(rk), ndv_R=len(set(rk)), f1_R=0, n_S=len(sk), ndv_S=len(set(sk)),
                       f1_S=0)
            expect += prob * Fraction(oe.join_estimate(res, 6, rr, 6, rs)["join_ht"])
    assert float(expect) == pytest.approx(truth, rel=1e-12)


def test_gee_closed_forms_and_error_bound():
    assert oe.gee(1000, 1000, 37, 5) == 37                       # whole table sampled: the exact NDV
    assert oe.gee(10_000, 100, 100, 100) == pytest.approx(1000)  # all singletons: sqrt(n/r) d
    assert oe.gee(10_000, 100, 20, 0) == 20                      # no singletons: d
    assert oe.gee(10_000, 0, 0, 0) == 0
    rng = np.random.default_rng(4)
    for s, n, r in [(1.1, 200_000, 2_000), (2.0, 100_000, 5_000), (0.0, 50_000, 500)]:
        col = (rng.zipf(s, n) if s else rng.integers(0, 30_000, n)).astype(np.int64)
        D = np.unique(col).size
        samp = rng.choice(col, r, replace=False)
        _, f = np.unique(samp, return_counts=True)
        est = oe.gee(n, r, f.size, int((f == 1).sum()))
        bound = math.e * math.sqrt(n / r)                        # GEE's ratio-error guarantee, loosened
        assert D / bound <= est <= D * bound


def test_selectivity_library_equals_oracle():
    rng = random.Random(3)
    for _ in range(5000):
        n = rng.choice([rng.randint(0, 50), rng.randint(0, 2**40)])
        s = rng.randint(0, n)
        c = rng.randint(0, s)
        rate = rng.choice([0.0, 1.0, rng.random(), 1e-6, 0.5])
        got = g.gace_estimate_selectivity(c, s, 0, n, rate)
        want = oe.sel_estimate(c, s, n, rate)
        for k in want:
            assert (math.isnan(got[k]) and math.isnan(want[k])) or got[k] == want[k], (k, c, s, n, rate)
    # at rate 1 the cardinality is the count itself
    assert g.gace_estimate_selectivity(17, 100, 1, 100, 1.0)["card_ht"] == 17


def test_join_library_equals_oracle():
    rng = random.Random(8)
    for _ in range(3000):
        nr, ns = rng.randint(0, 10**9), rng.randint(0, 10**9)
        res = {}
        for side, n in (("R", nr), ("S", ns)):
            m = rng.randint(0, min(n, 10**7))
            d = rng.randint(0, m)
            f1 = rng.randint(0, d)
            f2 = rng.randint(0, d - f1)
            res.update({"n_" + side: m, "ndv_" + side: d, "f1_" + side: f1, "f2_" + side: f2})
        res["join_card"] = rng.randint(0, 10**12)
        rr, rs = rng.choice([1.0, rng.random(), 0.0]), rng.choice([1.0, rng.random()])
        got = g.gace_estimate_join(res, nr, rr, ns, rs)
        want = oe.join_estimate(res, nr, rr, ns, rs)
        for k in want:
            assert (math.isnan(got[k]) and math.isnan(want[k])) or got[k] == want[k], k


def test_estimates_reject_impossible_counts():
    with pytest.raises(g.GaceError):
        g.gace_estimate_selectivity(5, 4, 1, 10)
    with pytest.raises(g.GaceError):
        g.gace_estimate_selectivity(1, 11, 1, 10)
    bad = dict(join_card=0, n_R=5, ndv_R=6, f1_R=0, f2_R=0, n_S=0, ndv_S=0, f1_S=0, f2_S=0)
    with pytest.raises(g.GaceError):
        g.gace_estimate_join(bad, 10, 1.0, 10, 1.0)
