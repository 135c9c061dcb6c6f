"""Pins of the CPU oracle against things other than itself: hand-worked
examples, library routines (numpy masks, np.unique, brute-force pair counts),
closed forms and invariants.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_probe.json")
OPS = {"RANGE": oracle.RANGE, "EQ": oracle.EQ, "IN": oracle.IN}
INT32_MIN, INT32_MAX = -(2**31), 2**31 - 1
INT64_MIN, INT64_MAX = -(2**63), 2**63 - 1


def _bits_to_f32(b):
    return float(np.array([b], dtype=np.uint32).view(np.float32)[0])


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _golden_table(g):
    s = g["selectivity"]
    c0 = np.array(s["c0_i32"], dtype=np.int32)
    c1 = np.array([int(x) for x in s["c1_i64"]], dtype=np.int64)
    c2 = np.array([int(x, 16) for x in s["c2_f32_bits"]], dtype=np.uint32).view(np.float32)
    return [c0, c1, c2], s["dtypes"]


def _golden_preds(g):
    preds = []
    for p in g["selectivity"]["predicates"]:
        terms = []
        for col, op, vals in p["terms"]:
            if col == 2:
                vv = tuple(_bits_to_f32(int(v, 16)) for v in vals)
            else:
                vv = tuple(int(v) for v in vals)
            terms.append((col, OPS[op], vv))
        preds.append(terms)
    return preds


# ---------------------------------------------------------------- hand-worked
def test_golden_selectivity_counts(golden):
    cols, dtypes = _golden_table(golden)
    preds = _golden_preds(golden)
    counts, sampled, kept = oracle.probe_selectivity(cols, dtypes, 9, preds, 123, 1.0, 4)
    expect = [p["count"] for p in golden["selectivity"]["predicates"]]
    assert counts.tolist() == expect
    assert sampled == 12 and kept == 3


def test_golden_joins(golden):
    for j in golden["joins"]:
        r = np.array([int(x) for x in j["R"]], dtype=np.int64)
        s = np.array([int(x) for x in j["S"]], dtype=np.int64)
        out = oracle.join_freq(r, 1, 5, 1.0, 4096, s, 2, 6, 1.0, 4096)
        for k in ("join_card", "ndv_R", "ndv_S", "n_R", "n_S"):
            assert out[k] == j[k], (k, j["why"])


def test_golden_thresholds(golden):
    for t in golden["thresholds"]:
        assert oracle.threshold(t["rate"]) == t["thr"], t["why"]


# ---------------------------------------------------------------- sampler
def test_rate_one_and_zero():
    n = 100_003
    assert oracle.kept_blocks(n, 77, 3, 1.0, 64).tolist() == list(range((n + 63) // 64))
    assert oracle.kept_blocks(n, 77, 3, 0.0, 64).size == 0


def test_sampler_nesting_by_rate():
    # same (seed, table): a block kept at a lower rate is kept at every higher rate
    n, B = 4_000_000, 256
    prev = None
    for rate in [0.001, 0.01, 0.05, 0.2, 0.5, 0.9, 1.0]:
        k = set(oracle.kept_blocks(n, 0xABCDEF, 11, rate, B).tolist())
        if prev is not None:
            assert prev <= k
        prev = k


@pytest.mark.parametrize("rate", [0.001, 0.01, 0.05, 0.3, 0.77])
def test_sampler_binomial(rate):
    # kept-block count ~ Binomial(nb, thr / 2^32): within 6 sigma
    nb = 200_000
    p = oracle.threshold(rate) / 2**32
    k = oracle.kept_blocks(nb, 0x5EED + int(rate * 1000), 4, rate, 1).size
    mu, sd = nb * p, math.sqrt(nb * p * (1 - p))
    assert abs(k - mu) <= 6 * sd


def test_philox_word0_uniform_chi2():
    # word 0 over 2^16 consecutive counters, binned on its top 8 bits
    L = oracle.lib()
    words = np.empty(65536, dtype=np.uint32)
    key = np.array([0x1234, 0x5678], dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    for i in range(65536):
        ctr = np.array([i, 0, 7, 0], dtype=np.uint32)
        L.orc_philox4x32_10(ctr.ctypes.data, key.ctypes.data, out.ctypes.data)
        words[i] = out[0]
    hist = np.bincount(words >> 24, minlength=256)
    e = 65536 / 256
    chi2 = float(((hist - e) ** 2 / e).sum())
    # 255 dof: mean 255, sd ~22.6; 6 sigma
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)
    assert np.unique(words).size > 65000   # a bijection of the counter: few 32-bit collisions


def test_philox_avalanche():
    # flipping one counter bit changes about half of the 128 output bits
    flips = []
    for bit in range(32):
        for base in range(8):
            a = oracle.philox4x32_10([base * 977, 3, 5, 0], [11, 13])
            b = oracle.philox4x32_10([(base * 977) ^ (1 << bit), 3, 5, 0], [11, 13])
            flips.append(sum(bin(x ^ y).count("1") for x, y in zip(a, b)))
    m = float(np.mean(flips))
    assert 60 < m < 68


def test_keep_matches_threshold_definition():
    # keep(b) is word0 < thr: for a fixed block, kept exactly when rate*2^32 > word0
    seed, tid = 0xFEEDFACE12345678, 17
    for b in range(50):
        w0 = oracle.philox4x32_10([b & 0xFFFFFFFF, b >> 32, tid, 0], [seed & 0xFFFFFFFF, seed >> 32])[0]
        assert not oracle.block_kept(seed, tid, b, w0)
        assert oracle.block_kept(seed, tid, b, w0 + 1)


# ---------------------------------------------------------------- counts
def _np_term(col, dt, op, vals):
    if op == oracle.RANGE:
        return (col >= vals[0]) & (col < vals[1])
    m = np.zeros(col.shape[0], dtype=bool)
    for v in vals:
        m |= col == v
    return m


def _np_counts(cols, dtypes, preds, rowmask):
    wide = [c.astype(np.int64) if dt == 1 else c for c, dt in zip(cols, dtypes)]
    out = []
    for p in preds:
        m = rowmask.copy()
        for (ci, op, vals) in p:
            v = [np.float32(x) for x in vals] if dtypes[ci] == 3 else vals
            m &= _np_term(wide[ci], dtypes[ci], op, v)
        out.append(int(np.count_nonzero(m)))
    return out


def _edge_table(rng, n):
    c0 = rng.integers(-5, 6, size=n).astype(np.int32)
    c0[rng.random(n) < 0.05] = INT32_MIN
    c0[rng.random(n) < 0.05] = INT32_MAX
    c1 = rng.integers(-3, 4, size=n).astype(np.int64)
    c1[rng.random(n) < 0.05] = INT64_MIN
    c1[rng.random(n) < 0.05] = INT64_MAX
    c2 = rng.choice(np.array([-1.5, -0.0, 0.0, 0.25, 0.5, 1.0, np.nan, np.inf, -np.inf], dtype=np.float32), size=n)
    c3 = rng.integers(0, 1000, size=n).astype(np.int32)
    return [c0, c1, c2, c3], [1, 2, 3, 1]


def _random_edge_preds(rng, n_preds):
    pools = {0: [INT32_MIN, -5, -1, 0, 1, 5, INT32_MAX], 1: [INT64_MIN, -3, 0, 3, INT64_MAX],
             2: [-1.5, -0.0, 0.0, 0.25, 1.0, float("inf"), float("-inf")], 3: [0, 10, 500, 999, 1000]}
    preds = []
    for _ in range(n_preds):
        k = int(rng.integers(1, 5))
        terms = []
        for _ in range(k):
            c = int(rng.integers(0, 4))
            op = int(rng.integers(1, 4))
            pool = pools[c]
            if op == oracle.RANGE:
                a, b = rng.choice(len(pool), 2)
                terms.append((c, op, (pool[a], pool[b])))
            elif op == oracle.EQ:
                terms.append((c, op, (pool[int(rng.integers(len(pool)))],)))
            else:
                m = int(rng.integers(1, 9))
                terms.append((c, op, tuple(pool[int(i)] for i in rng.integers(0, len(pool), m))))
        preds.append(terms)
    return preds


@pytest.mark.parametrize("seed", range(6))
def test_counts_brute_force_vs_numpy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3 * 4096 + 17))
    cols, dtypes = _edge_table(rng, n)
    preds = _random_edge_preds(rng, 24)
    B = int(2 ** rng.integers(0, 9))
    rate = [1.0, 0.5, 0.13, 0.0][seed % 4]
    counts, sampled, kept = oracle.probe_selectivity(cols, dtypes, 5 + seed, preds, 99 + seed, rate, B)
    blocks = oracle.kept_blocks(n, 99 + seed, 5 + seed, rate, B)
    rowmask = np.zeros(n, dtype=bool)
    for b in blocks:
        rowmask[int(b) * B:min(n, (int(b) + 1) * B)] = True
    assert kept == blocks.size
    assert sampled == int(rowmask.sum())
    assert counts.tolist() == _np_counts(cols, dtypes, preds, rowmask)


def test_threads_do_not_change_counts():
    rng = np.random.default_rng(42)
    cols, dtypes = _edge_table(rng, 50_000)
    preds = _random_edge_preds(rng, 16)
    a = oracle.probe_selectivity(cols, dtypes, 3, preds, 5, 0.4, 128, nthreads=1)
    b = oracle.probe_selectivity(cols, dtypes, 3, preds, 5, 0.4, 128, nthreads=7)
    assert a[0].tolist() == b[0].tolist() and a[1:] == b[1:]


def test_closed_form_config1():
    # 10^6 rows of two independent U[0,1000) columns: P = 0.2 * 0.5; E = 100000, sd = 300
    w = datagen.config1()
    counts, sampled, kept = oracle.sel_request(w, 0)
    assert sampled == 1_000_000 and kept == 245
    assert abs(int(counts[0]) - 100_000) <= 1800


def test_invariants_conjunction_and_complement():
    rng = np.random.default_rng(7)
    n = 30_000
    c0 = rng.integers(-(2**31), 2**31, size=n, dtype=np.int64).astype(np.int32)
    c1 = rng.integers(0, 100, size=n).astype(np.int32)
    cols, dtypes = [c0, c1], [1, 1]
    lo, hi = -12345678, 987654321
    A = [(0, oracle.RANGE, (lo, hi))]
    Bp = [(1, oracle.RANGE, (10, 60))]
    preds = [A, Bp, A + Bp,
             [(0, oracle.RANGE, (INT32_MIN, lo))], [(0, oracle.RANGE, (hi, 2**31))],
             [(0, oracle.RANGE, (lo - 1000, hi + 1000))], [(0, oracle.RANGE, (hi, lo))]]
    c, sampled, _ = oracle.probe_selectivity(cols, dtypes, 1, preds, 3, 0.6, 64)
    assert c[2] <= c[0] and c[2] <= c[1]                      # conjunction <= each conjunct
    assert c[0] + c[3] + c[4] == sampled                      # [lo,hi) + [MIN,lo) + [hi,2^31) cover i32
    assert c[5] >= c[0]                                       # widening never lowers
    assert c[6] == 0                                          # empty range


def test_pcs_correlated_vs_independent():
    # Eq. 3: PCS = P(A,B) / (P(A) P(B)).  c1 = c0 + U{-50..50} tracks c0, so aligned
    # ranges on c0 and c1 give PCS >> 1.6; c3 and c4 are independent uniforms, PCS ~ 1
    t = datagen.config2_table(400_000)
    cols = datagen.host_table(t)
    dtypes = [c.dtype for c in t.cols]
    A, B = (0, oracle.RANGE, (100, 2000)), (1, oracle.RANGE, (100, 2000))
    C, D = (3, oracle.RANGE, (0, 300_000)), (4, oracle.RANGE, (0, 500_000))
    c, n, _ = oracle.probe_selectivity(cols, dtypes, 2, [[A], [B], [A, B], [C], [D], [C, D]], 1, 1.0, 4096)
    pcs_ab = (c[2] / n) / ((c[0] / n) * (c[1] / n))
    pcs_cd = (c[5] / n) / ((c[3] / n) * (c[4] / n))
    assert pcs_ab > 1.6
    assert abs(pcs_cd - 1.0) < 0.05


# ---------------------------------------------------------------- joins
def _np_join(r, s):
    ur, fr = np.unique(r, return_counts=True)
    us, fs = np.unique(s, return_counts=True)
    common, ir, is_ = np.intersect1d(ur, us, assume_unique=True, return_indices=True)
    return int((fr[ir].astype(np.uint64) * fs[is_].astype(np.uint64)).sum()), ur.size, us.size


@pytest.mark.parametrize("seed", range(4))
def test_join_brute_force_pairs(seed):
    rng = np.random.default_rng(100 + seed)
    r = rng.integers(-20, 20, size=int(rng.integers(0, 2000))).astype(np.int64)
    s = rng.integers(-20, 20, size=int(rng.integers(0, 2000))).astype(np.int64)
    r[rng.random(r.size) < 0.03] = INT64_MIN
    s[rng.random(s.size) < 0.03] = INT64_MAX
    out = oracle.join_freq(r, 1, 0, 1.0, 1, s, 2, 0, 1.0, 1)
    pairs = int((r[:, None] == s[None, :]).sum())            # nested-loop equi-join size
    assert out["join_card"] == pairs
    assert out["ndv_R"] == np.unique(r).size and out["ndv_S"] == np.unique(s).size
    assert out["n_R"] == r.size and out["n_S"] == s.size
    # frequency of frequencies: keys seen exactly once / twice, counted by numpy
    for side, x in (("R", r), ("S", s)):
        _, f = np.unique(x, return_counts=True)
        assert out["f1_" + side] == int((f == 1).sum()) and out["f2_" + side] == int((f == 2).sum())


def test_join_sampled_vs_numpy():
    rng = np.random.default_rng(5)
    r = rng.zipf(1.5, size=300_000).astype(np.int64)
    s = rng.integers(0, 5000, size=120_000).astype(np.int64)
    B = 512
    out = oracle.join_freq(r, 31, 8, 0.3, B, s, 32, 9, 0.6, B)
    kr = oracle.kept_blocks(r.size, 8, 31, 0.3, B)
    ks = oracle.kept_blocks(s.size, 9, 32, 0.6, B)
    rs = np.concatenate([r[int(b) * B:(int(b) + 1) * B] for b in kr])
    ss = np.concatenate([s[int(b) * B:(int(b) + 1) * B] for b in ks])
    j, nr, ns = _np_join(rs, ss)
    assert (out["join_card"], out["ndv_R"], out["ndv_S"], out["n_R"], out["n_S"]) == (j, nr, ns, rs.size, ss.size)


def test_join_special_cases():
    n = 10_000
    perm = np.random.default_rng(1).permutation(n).astype(np.int64)
    o = oracle.join_freq(perm, 1, 0, 1.0, 64, perm[::-1].copy(), 2, 0, 1.0, 64)
    assert o["join_card"] == n and o["ndv_R"] == n and o["ndv_S"] == n
    eq = np.full(777, -42, dtype=np.int64)
    o = oracle.join_freq(eq, 1, 0, 1.0, 64, eq[:100], 2, 0, 1.0, 64)
    assert o["join_card"] == 777 * 100 and o["ndv_R"] == 1 and o["ndv_S"] == 1
    o = oracle.join_freq(np.arange(50, dtype=np.int64), 1, 0, 1.0, 64,
                         np.arange(50, 90, dtype=np.int64), 2, 0, 1.0, 64)
    assert o["join_card"] == 0
    o = oracle.join_freq(np.zeros(0, dtype=np.int64), 1, 0, 1.0, 64, eq, 2, 0, 1.0, 64)
    assert o == dict(join_card=0, ndv_R=0, ndv_S=1, n_R=0, n_S=777, f1_R=0, f1_S=0, f2_R=0, f2_S=0)
    o = oracle.join_freq(np.array([5, 5, 7, 9, 9, 9], dtype=np.int64), 1, 0, 1.0, 64,
                         np.array([1, 2, 2], dtype=np.int64), 2, 0, 1.0, 64)
    assert (o["f1_R"], o["f2_R"], o["f1_S"], o["f2_S"]) == (1, 1, 1, 1)


def test_join_invariants():
    rng = np.random.default_rng(9)
    r = rng.zipf(1.2, size=50_000).astype(np.int64)
    s = rng.integers(0, 300, size=20_000).astype(np.int64)
    rr = oracle.join_freq(r, 1, 3, 0.5, 128, r, 1, 3, 0.5, 128)
    kr = oracle.kept_blocks(r.size, 3, 1, 0.5, 128)
    rs = np.concatenate([r[int(b) * 128:(int(b) + 1) * 128] for b in kr])
    _, f = np.unique(rs, return_counts=True)
    assert rr["join_card"] == int((f.astype(np.uint64) ** 2).sum())      # join(R,R) = sum f^2
    assert int(f.sum()) == rr["n_R"]                                      # sum f = sampled n
    a = oracle.join_freq(r, 1, 3, 0.5, 128, s, 2, 4, 0.7, 64)
    b = oracle.join_freq(s, 2, 4, 0.7, 64, r, 1, 3, 0.5, 128)
    assert a["join_card"] == b["join_card"] and a["ndv_R"] == b["ndv_S"]  # symmetric


def test_join_overflow_guard():
    big = np.zeros(1, dtype=np.int64)
    # n_R * n_S >= 2^64 cannot be formed with real arrays here; the guard is
    # exercised through the C entry point with a fake length and no data read
    L = oracle.lib()
    out = np.zeros(9, dtype=np.uint64)
    rc = L.orc_join_freq(big.ctypes.data, 2**33, 1, 0, 1.0, 64, big.ctypes.data, 2**31, 2, 0, 1.0, 64,
                         out.ctypes.data)
    assert rc == -3


def test_iid_join_and_ndv_expectations():
    # R Zipf(1.0) over N, S iid uniform over N: E[join | R] = n_R n_S / N and
    # Var[join | R] <= n_S (1/N)(1 - 1/N) sum f_R^2 (S is multinomial);
    # E[NDV_S] = N (1 - (1 - 1/N)^n_S), Var <= E.
    w = datagen.config3(rate=1.0, n_r=2_000_000, n_s=500_000, domain=100_000)
    o = oracle.join_request(w, 0)
    jr = w.joins[0]
    kr = datagen.host_column(jr.r.cols[0], jr.r.n_rows)
    _, fr = np.unique(kr, return_counts=True)
    N, nr, ns = 100_000, 2_000_000, 500_000
    mu = nr * ns / N
    # the multinomial's covariance terms are negative, so the diagonal bounds the variance
    var = ns * (1 / N) * (1 - 1 / N) * float((fr.astype(np.float64) ** 2).sum())
    assert abs(o["join_card"] - mu) <= 6 * math.sqrt(var)
    e_ndv_s = N * (1 - (1 - 1 / N) ** ns)
    assert abs(o["ndv_S"] - e_ndv_s) <= 6 * math.sqrt(e_ndv_s)
    assert o["ndv_R"] == fr.size and o["n_R"] == nr and o["n_S"] == ns


def test_sort_is_sorted_permutation():
    rng = np.random.default_rng(3)
    k = rng.integers(INT64_MIN, INT64_MAX, size=100_000, dtype=np.int64)
    k[:10] = [INT64_MIN, INT64_MAX, 0, -1, 1, INT64_MIN, 0, 0, INT64_MAX, -1]
    assert np.array_equal(oracle.sort_i64(k), np.sort(k))
