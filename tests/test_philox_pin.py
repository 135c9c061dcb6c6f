"""Pin of the sampler's random source against an independent implementation.

The block sampler keeps block b iff word 0 of Philox4x32-10 (Salmon, Moraes,
Dror, Shaw, SC'11) under key = seed and counter = (b lo, b hi, table_id, 0) is
below floor(rate * 2^32) (the reading of the paper's block-level sampling,
Sec. II-A item 5 and Sec. III-B).  The oracle's generator is compared here with
rocRAND's Philox4x32-10 engine, compiled from the ROCm image's source header
by `tests/philox_rocrand.cpp`; the oracle never includes that header.

Mapping onto the rocRAND engine (its public constructor):
  engine(seed, subsequence = table_id, offset = 4 * block)
  -> key = (seed lo, seed hi), counter = (block lo, block hi, table_id, 0),
     and its first four draws are output words 0..3 of that counter.
CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_bin(tmp_path_factory):
    if not os.path.exists(HEADER) or shutil.which("g++") is None:
        pytest.skip("rocRAND source header or g++ not available")
    out = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run(["g++", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "philox_rocrand.cpp"), "-o", out], check=True)
    return out


def _triples(n):
    """(seed, block, table_id): both seed halves non-zero, blocks past 2^32, table ids > 0, edge values."""
    rng = np.random.default_rng(0x9E3779B9)
    seeds = rng.integers(1, 2**63, size=n, dtype=np.uint64) | np.uint64(1 << 63) * rng.integers(0, 2, size=n).astype(np.uint64)
    blocks = rng.integers(0, 2**40, size=n, dtype=np.uint64)
    blocks[: n // 4] = rng.integers(0, 1 << 20, size=n // 4, dtype=np.uint64)        # small block indices
    tids = rng.integers(0, 2**32, size=n, dtype=np.uint64)
    tids[: n // 8] = rng.integers(0, 64, size=n // 8, dtype=np.uint64)
    edge = [(0, 0, 0), (2**64 - 1, 0, 0), (0, 2**32 - 1, 0), (0, 2**32, 1), (2**64 - 1, 2**62 - 1, 2**32 - 1),
            (0x2512197500 + 32 + 2, 24414, 0), ((0xFFFFFFFF << 32) | 1, 1, 5), (1 << 32, 3, 7)]
    out = [(int(s), int(b), int(t)) for s, b, t in zip(seeds, blocks, tids)]
    return edge + out


def _rocrand_words(binary, triples):
    text = "".join("%d %d %d\n" % t for t in triples)
    res = subprocess.run([binary], input=text, capture_output=True, text=True, check=True)
    return [tuple(int(x, 16) for x in line.split()) for line in res.stdout.splitlines()]


def test_philox_all_words_match_rocrand(rocrand_bin):
    trip = _triples(100_000)
    ref = _rocrand_words(rocrand_bin, trip)
    assert len(ref) == len(trip)
    bad = []
    for (seed, block, tid), want in zip(trip, ref):
        got = oracle.philox4x32_10([block & 0xFFFFFFFF, block >> 32, tid, 0], [seed & 0xFFFFFFFF, seed >> 32])
        if tuple(got) != want:
            bad.append(((seed, block, tid), got, want))
            if len(bad) > 5:
                break
    assert not bad, bad


def test_block_decision_matches_rocrand_word0(rocrand_bin):
    # keep(b) = word0 < thr: the oracle's decision at thresholds on both sides of
    # rocRAND's word 0, and at the rates the workloads use
    trip = _triples(20_000)
    ref = _rocrand_words(rocrand_bin, trip)
    thrs = [oracle.threshold(r) for r in (0.001, 0.01, 0.05, 0.5)]
    for (seed, block, tid), w in zip(trip, ref):
        w0 = w[0]
        assert not oracle.block_kept(seed, tid, block, w0)
        assert oracle.block_kept(seed, tid, block, w0 + 1)
        for thr in thrs:
            assert oracle.block_kept(seed, tid, block, thr) == (w0 < thr)
