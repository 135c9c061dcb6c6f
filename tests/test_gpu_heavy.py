"""Join keys that the per-join heavy-hitter table takes out of the
partitioning (counted per table slot, like the sentinel key): every result
equals the oracle's whatever the table holds.  Cases that reach the table's
edges: skew on one side only, key-sorted columns (the sample's spread runs
then see locally repeated keys), hot keys whose hashes compete for one table
slot, sides shorter than the sample or just longer, an empty side, and one
join twice in a batch (two tables)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

INT64_MIN = -(2**63)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2512_19750_amd as g
    torch.cuda.set_device(0)
    ctx = g.gace_create(0, 2 << 30)
    yield g, ctx, torch.device("cuda:0")
    g.gace_destroy(ctx)


def _finalizer(k: np.ndarray) -> np.ndarray:
    """The 64-bit MurmurHash3 finalizer, used here only to choose keys whose
    hashes share their low 10 bits (one heavy-table slot)."""
    x = k.astype(np.uint64)
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(33)
        x *= np.uint64(0xFF51AFD7ED558CCD)
        x ^= x >> np.uint64(33)
        x *= np.uint64(0xC4CEB9FE1A85EC53)
        x ^= x >> np.uint64(33)
    return x


def _keys(case: str, rng):
    if case == "skew_on_s":
        r = rng.integers(0, 2_000_000, 400_000, dtype=np.int64)
        s = (rng.zipf(1.1, 300_000) % 50_000).astype(np.int64)
    elif case == "sorted":
        r = np.sort((rng.zipf(1.3, 600_000) % 100_000).astype(np.int64))
        s = np.sort(rng.integers(0, 100_000, 200_000, dtype=np.int64))
    elif case == "slot_contest":
        cand = np.arange(1, 400_000, dtype=np.int64)
        slot = _finalizer(cand) & np.uint64(1023)
        same = cand[slot == slot[0]][:8]
        assert len(same) == 8
        # eight hot keys of one slot, with different counts, among a uniform tail
        r = np.concatenate([np.repeat(same, [9000, 7000, 5000, 3000, 2000, 1000, 500, 2]),
                            rng.integers(500_000, 900_000, 200_000, dtype=np.int64)])
        s = np.concatenate([np.repeat(same, [3, 5000, 1, 0, 700, 0, 9, 2000]),
                            rng.integers(500_000, 900_000, 50_000, dtype=np.int64)])
        rng.shuffle(r)
        rng.shuffle(s)
    elif case == "short_sides":
        r = rng.integers(0, 50, 4095, dtype=np.int64)
        s = rng.integers(0, 50, 4097, dtype=np.int64)
    elif case == "just_above_sample":
        r = (rng.zipf(1.2, 4097) % 3000).astype(np.int64)
        s = (rng.zipf(1.2, 4353) % 3000).astype(np.int64)
    elif case == "empty_s":
        r = (rng.zipf(1.2, 300_000) % 10_000).astype(np.int64)
        s = np.zeros(0, dtype=np.int64)
    elif case == "sentinel_heavy":
        r = (rng.zipf(1.2, 300_000) % 10_000).astype(np.int64)
        s = (rng.zipf(1.2, 100_000) % 10_000).astype(np.int64)
        r[rng.random(r.size) < 0.3] = INT64_MIN          # the sentinel value is the hottest key
        s[rng.random(s.size) < 0.1] = INT64_MIN
    else:
        raise ValueError(case)
    return r, s


CASES = ["skew_on_s", "sorted", "slot_contest", "short_sides", "just_above_sample", "empty_s", "sentinel_heavy"]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("rate,B", [(1.0, 4096), (0.5, 16)])
def test_heavy_cases_vs_oracle(env, case, rate, B):
    import torch
    g, ctx, dev = env
    rng = np.random.default_rng(100 * CASES.index(case) + int(rate * 10) + B)
    r, s = _keys(case, rng)
    _say("heavy case", case, r.size, s.size, rate, B)
    kr = torch.from_numpy(r).to(dev)
    ks = torch.from_numpy(s).to(dev)
    got = g.gace_join_freq(ctx, g.Keys(kr, 11, 101, rate, B), g.Keys(ks, 12, 103, rate, B))
    assert got == oracle.join_freq(r, 11, 101, rate, B, s, 12, 103, rate, B)


def test_same_join_twice_in_a_batch(env):
    """Two joins of one batch over the same keys: each builds its own table
    from its own sample, and both equal the oracle."""
    import torch
    g, ctx, dev = env
    rng = np.random.default_rng(77)
    r = (rng.zipf(1.1, 500_000) % 40_000).astype(np.int64)
    s = rng.integers(0, 40_000, 200_000, dtype=np.int64)
    kr = torch.from_numpy(r).to(dev)
    ks = torch.from_numpy(s).to(dev)
    reqs = [g.JoinRequest(g.Keys(kr, 21, 5, 1.0, 4096), g.Keys(ks, 22, 6, 1.0, 4096)),
            g.JoinRequest(g.Keys(kr, 21, 7, 0.3, 64), g.Keys(ks, 22, 8, 0.3, 64))]
    g.gace_batch_run(ctx, reqs)
    assert reqs[0].result() == oracle.join_freq(r, 21, 5, 1.0, 4096, s, 22, 6, 1.0, 4096)
    assert reqs[1].result() == oracle.join_freq(r, 21, 7, 0.3, 64, s, 22, 8, 0.3, 64)
