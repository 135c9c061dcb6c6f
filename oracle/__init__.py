"""CPU oracle for the GACE Measurement Engine probe (arXiv 2512.19750, Sec. III-B).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything here, and nothing here imports the product package.

The arithmetic lives in oracle.c (plain C, built with gcc); this module only
marshals numpy arrays and the predicate lists of the `datagen` recipes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

F32 = 3
RANGE, EQ, IN = 1, 2, 3

TERM_DTYPE = np.dtype([("col", "<u4"), ("op", "<u4"), ("n_vals", "<u4"), ("pad", "<u4"), ("v", "<i8", (8,))])


class OrcCol(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


def build() -> str:
    subprocess.run(["gcc", "-O2", "-Wall", "-fPIC", "-shared", "-o", LIB, os.path.join(HERE, "oracle.c"),
                    "-lm", "-lpthread"], check=True)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        u32, u64, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_threshold.argtypes = [dbl]
        L.orc_threshold.restype = u64
        L.orc_block_kept.argtypes = [u64, u32, u64, u64]
        L.orc_block_kept.restype = ctypes.c_int
        L.orc_kept_blocks.argtypes = [u64, u64, u32, dbl, u32, P, u64]
        L.orc_kept_blocks.restype = u64
        L.orc_probe_selectivity.argtypes = [u64, P, u32, u32, P, P, u32, u64, dbl, u32, P, P, P, ctypes.c_int]
        L.orc_probe_selectivity.restype = ctypes.c_int
        L.orc_join_freq.argtypes = [P, u64, u32, u64, dbl, u32, P, u64, u32, u64, dbl, u32, P]
        L.orc_join_freq.restype = ctypes.c_int
        L.orc_sort_i64.argtypes = [P, u64]
        L.orc_sort_i64.restype = ctypes.c_int
        _lib = L
    return _lib


def _f32_bits(x) -> int:
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


def encode_predicates(preds, dtypes: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Predicate lists -> (orc_term array, uint32 offsets with n_preds + 1 entries)."""
    n_terms = sum(len(p) for p in preds)
    terms = np.zeros(max(n_terms, 1), dtype=TERM_DTYPE)
    off = np.zeros(len(preds) + 1, dtype=np.uint32)
    k = 0
    for i, p in enumerate(preds):
        for (col, op, vals) in p:
            terms[k]["col"] = col
            terms[k]["op"] = op
            terms[k]["n_vals"] = len(vals)
            for j, v in enumerate(vals):
                terms[k]["v"][j] = _f32_bits(v) if dtypes[col] == F32 else int(v)
            k += 1
        off[i + 1] = k
    return terms, off


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return tuple(int(x) for x in o)


def threshold(rate: float) -> int:
    return int(lib().orc_threshold(float(rate)))


def block_kept(seed: int, table_id: int, block: int, thr: int) -> bool:
    return bool(lib().orc_block_kept(seed, table_id, block, thr))


def kept_blocks(n_rows: int, seed: int, table_id: int, rate: float, block_rows: int) -> np.ndarray:
    nb = (n_rows + block_rows - 1) // block_rows
    out = np.empty(max(nb, 1), dtype=np.uint64)
    k = lib().orc_kept_blocks(n_rows, seed, table_id, float(rate), block_rows, out.ctypes.data, nb)
    return out[:k].copy()


def probe_selectivity(cols: List[np.ndarray], dtypes: Sequence[int], table_id: int, preds,
                      seed: int, rate: float, block_rows: int, nthreads: int = 8):
    """-> (counts uint64[n_preds], sampled_rows, kept_blocks)."""
    n_rows = int(cols[0].shape[0]) if cols else 0
    arr = (OrcCol * max(len(cols), 1))()
    keep = []
    for i, (c, dt) in enumerate(zip(cols, dtypes)):
        c = np.ascontiguousarray(c)
        keep.append(c)
        arr[i].data = c.ctypes.data
        arr[i].dtype = dt
    terms, off = encode_predicates(preds, dtypes)
    counts = np.zeros(max(len(preds), 1), dtype=np.uint64)
    sampled = ctypes.c_uint64()
    kept = ctypes.c_uint64()
    rc = lib().orc_probe_selectivity(n_rows, ctypes.addressof(arr), len(cols), table_id, terms.ctypes.data,
                                     off.ctypes.data, len(preds), seed, float(rate), block_rows,
                                     counts.ctypes.data, ctypes.addressof(sampled), ctypes.addressof(kept),
                                     nthreads)
    if rc != 0:
        raise ValueError("orc_probe_selectivity rejected its arguments (%d)" % rc)
    return counts[:len(preds)], int(sampled.value), int(kept.value)


def join_freq(keys_r: np.ndarray, tid_r: int, seed_r: int, rate_r: float, br: int,
              keys_s: np.ndarray, tid_s: int, seed_s: int, rate_s: float, bs: int) -> Dict[str, int]:
    keys_r = np.ascontiguousarray(keys_r, dtype=np.int64)
    keys_s = np.ascontiguousarray(keys_s, dtype=np.int64)
    out = np.zeros(9, dtype=np.uint64)
    rc = lib().orc_join_freq(keys_r.ctypes.data, keys_r.shape[0], tid_r, seed_r, float(rate_r), br,
                             keys_s.ctypes.data, keys_s.shape[0], tid_s, seed_s, float(rate_s), bs,
                             out.ctypes.data)
    if rc == -3:
        raise OverflowError("n_R * n_S >= 2^64")
    if rc != 0:
        raise ValueError("orc_join_freq rejected its arguments (%d)" % rc)
    return dict(join_card=int(out[0]), ndv_R=int(out[1]), ndv_S=int(out[2]), n_R=int(out[3]), n_S=int(out[4]),
                f1_R=int(out[5]), f1_S=int(out[6]), f2_R=int(out[7]), f2_S=int(out[8]))


def sort_i64(keys: np.ndarray) -> np.ndarray:
    k = np.array(keys, dtype=np.int64, copy=True)
    if lib().orc_sort_i64(k.ctypes.data, k.shape[0]) != 0:
        raise MemoryError
    return k


# ----------------------------------------------------------------------------
# workload helpers: regenerate only the kept blocks, then count on them
# ----------------------------------------------------------------------------
def _kept_rows(n_rows: int, blocks: np.ndarray, block_rows: int) -> List[Tuple[int, int]]:
    return [(int(b) * block_rows, min(n_rows, (int(b) + 1) * block_rows)) for b in blocks]


def sel_request(w, i: int, nthreads: int = 8):
    """Oracle result of selectivity request i of a datagen Workload:
    the kept blocks come from the oracle's sampler, their rows are regenerated
    on the host, and the predicates are counted on those rows."""
    import datagen
    req = w.sel[i]
    t = w.tables[req.table]
    sp = req.spec
    blocks = kept_blocks(t.n_rows, sp.seed, t.table_id, sp.rate, sp.block_rows)
    spans = _kept_rows(t.n_rows, blocks, sp.block_rows)
    dtypes = [c.dtype for c in t.cols]
    if not spans:
        return np.zeros(len(req.preds), dtype=np.uint64), 0, 0
    full = len(spans) == (t.n_rows + sp.block_rows - 1) // sp.block_rows
    if full:
        cols = datagen.host_table(t, nthreads=nthreads)
    else:
        cols = []
        for c in t.cols:
            parts = [datagen.host_column(c, e - b, row0=b, nthreads=nthreads) for b, e in merge_spans(spans)]
            cols.append(np.concatenate(parts))
    counts, sampled, _ = probe_selectivity(cols, dtypes, t.table_id, req.preds, 0, 1.0, 1 << 20, nthreads)
    return counts, sampled, len(spans)


def merge_spans(spans):
    out = []
    for b, e in spans:
        if out and out[-1][1] == b:
            out[-1] = (out[-1][0], e)
        else:
            out.append((b, e))
    return out


def sampled_keys(t, spec, nthreads: int = 8) -> np.ndarray:
    import datagen
    blocks = kept_blocks(t.n_rows, spec.seed, t.table_id, spec.rate, spec.block_rows)
    spans = merge_spans(_kept_rows(t.n_rows, blocks, spec.block_rows))
    if not spans:
        return np.zeros(0, dtype=np.int64)
    return np.concatenate([datagen.host_column(t.cols[0], e - b, row0=b, nthreads=nthreads) for b, e in spans])


def join_request(w, j: int, nthreads: int = 8) -> Dict[str, int]:
    """Oracle result of join request j: kept key blocks regenerated on the host,
    then the sort-based frequency join over them (rate 1)."""
    jr = w.joins[j]
    kr = sampled_keys(jr.r, jr.spec_r, nthreads)
    ks = sampled_keys(jr.s, jr.spec_s, nthreads)
    return join_freq(kr, jr.r.table_id, 0, 1.0, 1 << 20, ks, jr.s.table_id, 0, 1.0, 1 << 20)
